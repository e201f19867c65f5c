// One launch for the whole pass sequence of Algorithm 1 over frames of one
// size: a persistent grid of co-resident workgroups takes work items from
// one queue and runs each with the row-pass or column-pass body of the
// per-pass kernels (ils_passes.hpp), so the results are bitwise those of
// the per-pass launches.
//
// Work items, in queue order: for each pass p = 0 .. 2N (p = 0 the first
// row pass, odd p the column passes, even p the middle row passes, p = 2N
// the final row pass), for each unit (frame, channel) in order, the unit's
// bands (row passes) or column tiles.  An item of pass p > 0 of a unit
// waits until every item of pass p - 1 of that unit has completed: a row
// pass needs all columns of its channel transformed (and reads halo rows
// written by other bands' column tiles), a column pass needs all rows.
// These per-unit dependencies let the passes of one channel run beside
// those of the next, and remove the launch gaps between passes.
//
// Progress: tickets are handed out by one atomic counter in queue order, and
// an item only waits on items with smaller tickets, which running
// workgroups hold; so some item can always proceed.  Every wait is bounded
// in time (the real-time clock): on expiry the workgroup records an error
// flag and goes on (the results are then undefined, the kernel still ends),
// which the host reports; once the flag is set, every other wait gives up
// too.  No memory index depends on the data, so a run that gave up still
// stays in bounds.
//
// Memory ordering across the accelerator dies (each has its own L2): a
// finished item's workgroup makes its stores visible at device scope (every
// wave waits for its stores, then one thread issues a device-scope release
// fence and a relaxed atomic increment of the unit's counter); a waiting
// workgroup polls the counter with device-scope loads and issues a
// device-scope acquire fence before any of its threads reads the data.
#pragma once

#include "ils_launch.hpp"

namespace ilsk {

// Per-launch control block in device memory, zeroed by k_persist_reset before
// every launch: [0] ticket counter (alone in its 128-byte line), from
// [kPersistCtlHead] one completion counter per (pass, unit).  err: a word
// outside it that a wait which gave up sets to 1 (read and cleared by the
// host).
struct PersistList {
  const FrameDesc* descs;  // device array, n frames (all of one size)
  FrameDesc one;           // the frame when descs == nullptr
  int* ctl;                // control block: 2 + (2N + 1) * units ints
  int* err;
  const int* ch_start;     // device array, n + 1 prefix sums of the frames'
                           // channel counts; nullptr: every frame has C
  int n, C, N;
  int first;               // ROW_FIRST or ROW_FIRST_SAME
  int nb_row, nb_col;      // bands and column tiles per unit
  long long wait_ticks;    // real-time clock ticks (100 MHz) before a wait gives up
};

constexpr int kPersistCtlHead = 32;

template <int = 0>
__global__ void k_persist_reset(int* ctl, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) ctl[i] = 0;
}

template <int Pr, int Qr, int G, int Pc, int Qc, int S>
struct PersistCfg {
  static constexpr int RT = RowCfg<Pr, Qr, G>::THREADS;
  static constexpr int CT = ColCfg<Pc, Qc, S>::THREADS;
  static constexpr int THREADS = RT > CT ? RT : CT;
  static constexpr int RL = RowCfg<Pr, Qr, G>::LDS_F;
  static constexpr int CL = ColCfg<Pc, Qc, S>::LDS_F;
  static constexpr int LDS_F = RL > CL ? RL : CL;
  static constexpr int WAVES = waves_per_simd(THREADS, 4 * LDS_F);
};

template <int Pr, int Qr, int G, int Pc, int Qc, int S, int PEN>
__global__ void __launch_bounds__((PersistCfg<Pr, Qr, G, Pc, Qc, S>::THREADS))
__attribute__((amdgpu_waves_per_eu(PersistCfg<Pr, Qr, G, Pc, Qc, S>::WAVES))) k_persist(PersistList fl) {
  using Cfg = PersistCfg<Pr, Qr, G, Pc, Qc, S>;
  __shared__ float smem[Cfg::LDS_F];
  __shared__ int sh_ticket;
  ILS_G int* ctl = gm(fl.ctl);
  const int units = fl.ch_start ? gm(fl.ch_start)[fl.n] : fl.n * fl.C;
  const int npass = 2 * fl.N + 1;
  const long long row_items = (long long)units * fl.nb_row;
  const long long col_items = (long long)units * fl.nb_col;
  // passes 0, 2, ..., 2N are row passes; 1, 3, ..., 2N - 1 column passes
  const long long total = (long long)(fl.N + 1) * row_items + (long long)fl.N * col_items;
  const int tid = threadIdx.x;
  for (;;) {
    if (tid == 0) sh_ticket = __hip_atomic_fetch_add(ctl, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const long long t = sh_ticket;
    __syncthreads();  // every thread has read the ticket before thread 0 takes the next
    if (t >= total) break;
    // decode: a pair of passes (row, column) holds row_items + col_items tickets
    const long long pair = t / (row_items + col_items);
    long long rem = t - pair * (row_items + col_items);
    int p = (int)(2 * pair);
    int nb = fl.nb_row;
    if (rem >= row_items) {
      rem -= row_items;
      p += 1;
      nb = fl.nb_col;
    }
    const int unit = (int)(rem / nb);
    const int local = (int)(rem - (long long)unit * nb);
    int frame, ch;
    if (fl.ch_start) {
      frame = __builtin_amdgcn_readfirstlane(find_frame(gm(fl.ch_start), fl.n, unit));
      ch = unit - gm(fl.ch_start)[frame];
    } else {
      frame = unit / fl.C;
      ch = unit - frame * fl.C;
    }
    if (p > 0) {
      if (tid == 0) {
        const ILS_G int* cnt = ctl + kPersistCtlHead + (p - 1) * units + unit;
        const int need = (p & 1) ? fl.nb_row : fl.nb_col;  // items of pass p - 1
        // The wait is bounded in time by the constant-rate real-time clock
        // (not by a count of polls, whose latency has no bound under
        // contention); it also gives up as soon as another wait has given up
        // (checked every 16 polls), and at once if one already has.
        const unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
        int polls = 0;
        bool give_up = __hip_atomic_load(gm(fl.err), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
        while (!give_up && __hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
          __builtin_amdgcn_s_sleep(8);
          ++polls;
          give_up = (__builtin_amdgcn_s_memrealtime() - t0) > (unsigned long long)fl.wait_ticks ||
                    ((polls & 15) == 0 && __hip_atomic_load(gm(fl.err), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        }
        if (give_up) __hip_atomic_store(gm(fl.err), 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      }
      __syncthreads();
    }
    const FrameDesc d = fl.descs ? FrameDesc(gm(fl.descs)[frame]) : fl.one;
    if (p & 1) {
      col_body<Pc, Qc, S>(d, local, ch, smem);
    } else if (p == npass - 1) {
      row_final_body<Pr, Qr, G>(d, local, ch, smem);
    } else if (p == 0) {
      if (fl.first == ROW_FIRST_SAME)
        row_body<Pr, Qr, G, ROW_FIRST_SAME, PEN>(d, local, ch, smem);
      else
        row_body<Pr, Qr, G, ROW_FIRST, PEN>(d, local, ch, smem);
    } else {
      row_body<Pr, Qr, G, ROW_MID, PEN>(d, local, ch, smem);
    }
    // every wave waits until its stores have reached its die's L2; then one
    // device-scope release (write-back of that L2) and one increment for the
    // workgroup
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (tid == 0) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __hip_atomic_fetch_add(ctl + kPersistCtlHead + p * units + unit, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// Host-side entry of one persistent (row length, column length) pair.
struct PersistOps {
  int M, H;       // row complex length W/2 and column length
  int rows, cols; // band height and column-tile width (as the per-pass shapes)
  int threads, lds_bytes;
  // launches the reset and the persistent grid (grid = 0: co-resident count)
  hipError_t (*launch)(int pen, const PersistList& fl, int ctl_ints, int grid, hipStream_t st);
  // co-resident workgroups per CU of the instance for penalty pen
  int (*per_cu)(int pen);
};

template <int Pr, int Qr, int G, int Pc, int Qc, int S, int PEN>
int persist_per_cu_one() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_persist<Pr, Qr, G, Pc, Qc, S, PEN>,
                                                   PersistCfg<Pr, Qr, G, Pc, Qc, S>::THREADS, 0) != hipSuccess)
    return 0;
  return nb;
}

template <int Pr, int Qr, int G, int Pc, int Qc, int S>
int persist_per_cu(int pen) {
  static const int nc = persist_per_cu_one<Pr, Qr, G, Pc, Qc, S, PEN_CHARBONNIER>();
  static const int nw = persist_per_cu_one<Pr, Qr, G, Pc, Qc, S, PEN_WELSCH>();
  return pen == PEN_WELSCH ? nw : nc;
}

template <int Pr, int Qr, int G, int Pc, int Qc, int S>
hipError_t launch_persist(int pen, const PersistList& fl, int ctl_ints, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_persist_reset<>, dim3((ctl_ints + 255) / 256), dim3(256), 0, st, fl.ctl, ctl_ints);
  const dim3 block(PersistCfg<Pr, Qr, G, Pc, Qc, S>::THREADS);
  if (pen == PEN_WELSCH)
    hipLaunchKernelGGL((k_persist<Pr, Qr, G, Pc, Qc, S, PEN_WELSCH>), dim3(grid), block, 0, st, fl);
  else
    hipLaunchKernelGGL((k_persist<Pr, Qr, G, Pc, Qc, S, PEN_CHARBONNIER>), dim3(grid), block, 0, st, fl);
  return hipGetLastError();
}

template <int Pr, int Qr, int G, int Pc, int Qc, int S>
PersistOps make_persist() {
  using C = PersistCfg<Pr, Qr, G, Pc, Qc, S>;
  return PersistOps{Pr * Qr, Pc * Qc, G, S, C::THREADS, 4 * C::LDS_F, &launch_persist<Pr, Qr, G, Pc, Qc, S>,
                  &persist_per_cu<Pr, Qr, G, Pc, Qc, S>};
}

}  // namespace ilsk

// The persistent launch of one size: row length M = Pr * Qr with bands of G rows,
// column length H = Pc * Qc with tiles of S columns.
#define ILS_DEFINE_PERSIST(M, Pr, Qr, G, H, Pc, Qc, S)                          \
  const ilsk::PersistOps* ilsk_persist_##M##_##H() {                              \
    static const ilsk::PersistOps o = ilsk::make_persist<Pr, Qr, G, Pc, Qc, S>(); \
    return &o;                                                                \
  }
