// C ABI of the ILS library (declared in include/ils.h): argument validation,
// plan tables, workspace carve-up and the 2N+1 pass launch sequence of
// Algorithm 1 (first row pass, then N column passes interleaved with N-1
// middle row passes, then the final row pass).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <new>
#include <vector>

#include "../../include/ils.h"
#include "ils_persist.hpp"
#include "ils_launch.hpp"

using ilsk::WorkList;
using ilsk::cf;
using ilsk::FrameDesc;
using ilsk::ColVariant;
using ilsk::LenOps;
using ilsk::RowVariant;

// ---------------------------------------------------------------- registry
#define ILS_LEN(L, P, Q) const LenOps* ilsk_ops_##L();
#include "lengths.def"
#undef ILS_LEN
#define ILS_PERSIST(M, Pr, Qr, G, H, Pc, Qc, S) const ilsk::PersistOps* ilsk_persist_##M##_##H();
#include "persist.def"
#undef ILS_PERSIST

// Runtime-length passes (ils_generic.hip) for 2/3/5-smooth lengths up to
// kMaxGenericLen without a compiled split.
const LenOps* ilsk_generic_ops(int H);

namespace {

constexpr int kMaxGenericLen = 4096;

typedef const LenOps* (*OpsFn)();
const OpsFn kOps[] = {
#define ILS_LEN(L, P, Q) &ilsk_ops_##L,
#include "lengths.def"
#undef ILS_LEN
};
const int kLens[] = {
#define ILS_LEN(L, P, Q) L,
#include "lengths.def"
#undef ILS_LEN
};
constexpr int kNumLens = sizeof(kLens) / sizeof(kLens[0]);

const LenOps* find_ops(int L) {
  for (int i = 0; i < kNumLens; ++i)
    if (kLens[i] == L) return kOps[i]();
  return nullptr;
}

typedef const ilsk::PersistOps* (*PersistFn)();
const PersistFn kPersist[] = {
#define ILS_PERSIST(M, Pr, Qr, G, H, Pc, Qc, S) &ilsk_persist_##M##_##H,
#include "persist.def"
#undef ILS_PERSIST
};

// The persistent single-launch sequence for row length M and column length H, if
// one is compiled.
const ilsk::PersistOps* find_persist(int M, int H) {
  for (PersistFn fn : kPersist) {
    const ilsk::PersistOps* o = fn();
    if (o->M == M && o->H == H) return o;
  }
  return nullptr;
}

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

bool smooth235(int n) {
  if (n < 1) return false;
  while (n % 2 == 0) n /= 2;
  while (n % 3 == 0) n /= 3;
  while (n % 5 == 0) n /= 5;
  return n == 1;
}

// Lengths the runtime-length passes serve (no compiled split).
bool generic_length(int L) { return L >= 2 && L <= kMaxGenericLen && smooth235(L) && !find_ops(L); }

// Padded spectrum row length (complex elements): W/2+1 rounded up to 16
// (128-byte rows).
inline int spec_ld(int W) { return (int)align_up((size_t)(W / 2 + 1), 16); }

inline size_t frame_ws_bytes(int H, int W, int C) {
  return align_up(2ull * (size_t)C * (size_t)H * (size_t)spec_ld(W) * sizeof(cf), 256);
}

// Device-resident header of the workspace: batch work lists (descriptors and
// starts) from its start, the control blocks of persistent launches in its last
// kPersistCtlBytes, whose last 256 bytes hold the wait-expiry word.
constexpr size_t kBatchHeaderBytes = 1 << 20;
constexpr size_t kPersistCtlBytes = 256 << 10;
constexpr size_t kBatchListBytes = kBatchHeaderBytes - kPersistCtlBytes;
constexpr size_t kPersistErrOff = kBatchHeaderBytes - 256;
constexpr size_t kPersistCtlInts = (kPersistCtlBytes - 256) / sizeof(int);
// Time a wait of a persistent launch may take before it gives up, in ticks
// of the 100 MHz real-time clock: 20 ms.
constexpr long long kPersistWaitTicks = 2000000;
constexpr int kChains = 2;  // independent chains of passes in a batch graph
// Frames of at least this many pixel-channels fill the chip on their own:
// in a batch each is a part of its own (see ils_smooth_batch).
constexpr long long kPartPxCh = 1LL << 22;
constexpr int kMaxBatchFrames = 4096;
constexpr size_t kGraphCache = 4;  // batch graphs kept per plan

}  // namespace

// Per-length device tables (offsets into the plan's table buffer).
struct LenTables {
  size_t tw, tw2, sx, sy, twm;  // byte offsets
};

// Pinned host staging for the small host-to-device uploads (batch work
// lists, reduction jobs).  A slot is reused only after the copy that read it
// has completed (its event has fired).
constexpr int kStageSlots = 8;
constexpr size_t kStageBytes = kBatchHeaderBytes;

struct ils_plan {
  int max_H, max_W, max_C, max_frames;
  char* ws;
  size_t ws_bytes;
  hipStream_t stream;
  unsigned flags;
  int device;
  int last_error;
  char* tables;
  std::map<int, LenTables> tab;
  char* stage[kStageSlots];
  hipEvent_t stage_ev[kStageSlots];
  bool stage_used[kStageSlots];
  int stage_next;
  // graph of the last batched call (replayed while the batch structure repeats);
  // chain c > 0 of its passes is captured on chain_stream[c], forked from
  // cap_stream by fork_ev and joined back by join_ev[c]
  hipStream_t cap_stream;
  hipStream_t chain_stream[kChains];
  hipEvent_t fork_ev, join_ev[kChains];
  // a few graphs of recent batch structures, most recently used first
  // (gated surrogate inference alternates two structures per call)
  struct BatchGraph {
    std::vector<long long> sig;
    hipGraphExec_t exec;
  };
  std::vector<BatchGraph> graphs;
  // tile shapes chosen per image size (H, W, C) -> (row variant, column variant)
  std::map<long long, std::pair<int, int>> tuned;
  std::string arch;
  // pass timing
  bool prof_on;
  // persistent single-launch sequences (sizes of persist.def) on, and the device's
  // compute-unit count (grid of a persistent launch)
  bool persist_on;
  int cus;
  long long wait_ticks;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used;
  std::vector<int> prof_kind;  // kind of launch i; events 2i, 2i+1
};

// ----------------------------------------------------------------- helpers
static int record(ils_plan* plan, hipError_t e) {
  if (e == hipSuccess) return ILS_OK;
  if (plan && plan->last_error == ILS_OK) plan->last_error = (int)e;
  return ILS_ERR_HIP;
}

// Copy `bytes` of host data to device memory `dst` on the plan's stream via
// a pinned staging slot.
static hipError_t stage_upload(ils_plan* plan, void* dst, const void* src, size_t bytes) {
  if (bytes > kStageBytes) return hipErrorInvalidValue;
  const int s = plan->stage_next;
  plan->stage_next = (s + 1) % kStageSlots;
  if (plan->stage_used[s]) {
    hipError_t e = hipEventSynchronize(plan->stage_ev[s]);
    if (e != hipSuccess) return e;
  }
  std::memcpy(plan->stage[s], src, bytes);
  hipError_t e = hipMemcpyAsync(dst, plan->stage[s], bytes, hipMemcpyHostToDevice, plan->stream);
  if (e != hipSuccess) return e;
  e = hipEventRecord(plan->stage_ev[s], plan->stream);
  plan->stage_used[s] = (e == hipSuccess);
  return e;
}

// Launch wrapper: brackets the launch with timing events when profiling.
// kind: 0 first row, 1 middle row, 2 final row, 3 column.
template <class F>
static hipError_t timed(ils_plan* plan, int kind, F&& launch) {
  if (!plan->prof_on) return launch();
  while (plan->ev_pool.size() < plan->ev_used + 2) {
    hipEvent_t ev;
    hipError_t e = hipEventCreate(&ev);
    if (e != hipSuccess) return e;
    plan->ev_pool.push_back(ev);
  }
  hipEvent_t a = plan->ev_pool[plan->ev_used], b = plan->ev_pool[plan->ev_used + 1];
  hipError_t e = hipEventRecord(a, plan->stream);
  if (e != hipSuccess) return e;
  e = launch();
  if (e != hipSuccess) return e;
  e = hipEventRecord(b, plan->stream);
  if (e != hipSuccess) return e;
  plan->ev_used += 2;
  plan->prof_kind.push_back(kind);
  return hipSuccess;
}

static void free_plan(ils_plan* plan) {
  for (hipEvent_t ev : plan->ev_pool) (void)hipEventDestroy(ev);
  for (auto& g : plan->graphs) (void)hipGraphExecDestroy(g.exec);
  if (plan->cap_stream) (void)hipStreamDestroy(plan->cap_stream);
  for (int c = 1; c < kChains; ++c) {
    if (plan->chain_stream[c]) (void)hipStreamDestroy(plan->chain_stream[c]);
    if (plan->join_ev[c]) (void)hipEventDestroy(plan->join_ev[c]);
  }
  if (plan->fork_ev) (void)hipEventDestroy(plan->fork_ev);
  for (int i = 0; i < kStageSlots; ++i) {
    if (plan->stage_used[i]) (void)hipEventSynchronize(plan->stage_ev[i]);
    if (plan->stage_ev[i]) (void)hipEventDestroy(plan->stage_ev[i]);
    if (plan->stage[i]) (void)hipHostFree(plan->stage[i]);
  }
  if (plan->tables) (void)hipFree(plan->tables);
  delete plan;
}

static bool finite_f(float v) { return std::isfinite(v); }

static int check_params(float lambda, float p, float eps, int N) {
  if (!finite_f(lambda) || lambda < 0.0f) return ILS_ERR_INVALID_ARG;
  if (!finite_f(p) || !(p > 0.0f) || p > 2.0f) return ILS_ERR_INVALID_ARG;
  if (!finite_f(eps) || !(eps > 0.0f)) return ILS_ERR_INVALID_ARG;
  if (N < 0) return ILS_ERR_INVALID_ARG;
  return ILS_OK;
}

static int check_params_welsch(float lambda, float gamma, int N) {
  if (!finite_f(lambda) || lambda < 0.0f) return ILS_ERR_INVALID_ARG;
  if (!finite_f(gamma) || !(gamma > 0.0f)) return ILS_ERR_INVALID_ARG;
  if (N < 0) return ILS_ERR_INVALID_ARG;
  return ILS_OK;
}

static int check_frame_params(const ils_frame& fr) {
  if (fr.penalty == ILS_PENALTY_WELSCH) return check_params_welsch(fr.lambda, fr.gamma, fr.N);
  if (fr.penalty != ILS_PENALTY_CHARBONNIER) return ILS_ERR_INVALID_ARG;
  return check_params(fr.lambda, fr.p, fr.eps, fr.N);
}

static int check_size(const ils_plan* plan, int H, int W, int C) {
  if (H < 2 || W < 2 || C < 1) return ILS_ERR_INVALID_ARG;
  if (plan && (H > plan->max_H || W > plan->max_W || C > plan->max_C)) return ILS_ERR_INVALID_ARG;
  if (!ils_size_supported(H, W)) return ILS_ERR_UNSUPPORTED_SIZE;
  return ILS_OK;
}

// Fill a descriptor for one frame; the caller sets f/u0/out and the
// spectrum pointers.
static void fill_desc_on(const char* tables, const std::map<int, LenTables>& tab, FrameDesc& d, int H, int W,
                         int C, float lambda, float p, float eps) {
  const double c0 = (double)p * std::pow((double)eps, (double)p / 2.0 - 1.0);  // Eq. (11)
  const int M = W / 2;
  const LenTables& tr = tab.at(M);
  const LenTables& tc = tab.at(H);
  d.tw_row = reinterpret_cast<const cf*>(tables + tr.tw);
  d.tw2_row = reinterpret_cast<const cf*>(tables + tr.tw2);
  d.twm_row = reinterpret_cast<const cf*>(tables + tr.twm);
  d.sx = reinterpret_cast<const float*>(tables + tr.sx);
  d.tw_col = reinterpret_cast<const cf*>(tables + tc.tw);
  d.twm_col = reinterpret_cast<const cf*>(tables + tc.twm);
  d.sy = reinterpret_cast<const float*>(tables + tc.sy);
  d.H = H;
  d.W = W;
  d.C = C;
  d.ldS = spec_ld(W);
  d.kappa = (float)((double)lambda * c0 / 2.0);
  d.a_exp = (float)((double)p / 2.0 - 1.0);
  d.inv_eps = (float)(1.0 / (double)eps);
  d.log2_r = 0.0f;
  d.col_scale = (float)(1.0 / (2.0 * (double)H * (double)W));
  d.boost = 0.0f;
  d.nb_row = 0;
}
static void fill_desc(const ils_plan* plan, FrameDesc& d, int H, int W, int C, float lambda, float p, float eps) {
  fill_desc_on(plan->tables, plan->tab, d, H, W, C, lambda, p, eps);
}

// Welsch penalty (Sec. 5): c = c0 = 2 (Eq. (20)), so kappa = lambda; the
// pointwise step takes w = -log2(e) / (2 gamma^2).
static void fill_desc_welsch(const ils_plan* plan, FrameDesc& d, int H, int W, int C, float lambda,
                             float gamma) {
  fill_desc(plan, d, H, W, C, 1.0f, 1.0f, 1.0f);
  const double g = (double)gamma;
  d.kappa = lambda;
  d.a_exp = (float)(-1.4426950408889634 / (2.0 * g * g));
  d.inv_eps = 0.0f;
  d.log2_r = 0.0f;
}

// Tables of every compiled length, computed in double and rounded once to
// float: twiddles, real-FFT factors, the |F(nabla)|^2 eigenvalues of the
// periodic [1,-1] kernel (Eq. (9)) and the twiddle matrices of the
// four-step split.  Offsets into `host` (256-byte aligned) go to `tab`.
static void build_tables(std::vector<char>& host, std::map<int, LenTables>& tab) {
  auto put = [&](size_t bytes) {
    size_t off = align_up(host.size(), 256);
    host.resize(off + bytes);
    return off;
  };
  for (int i = 0; i < kNumLens; ++i) {
    const int L = kLens[i];
    LenTables t;
    t.tw = put(sizeof(cf) * L);
    t.tw2 = put(sizeof(cf) * (L + 1));
    t.sx = put(sizeof(float) * (L + 1));
    t.sy = put(sizeof(float) * L);
    cf* tw = reinterpret_cast<cf*>(host.data() + t.tw);
    for (int j = 0; j < L; ++j) {
      double a = -2.0 * M_PI * (double)j / (double)L;
      tw[j] = cf{(float)std::cos(a), (float)std::sin(a)};
    }
    cf* tw2 = reinterpret_cast<cf*>(host.data() + t.tw2);
    for (int k = 0; k <= L; ++k) {
      double a = -M_PI * (double)k / (double)L;
      tw2[k] = cf{(float)std::cos(a), (float)std::sin(a)};
    }
    // |F(nabla)|^2 for the periodic [1,-1] kernel: 4 sin^2(pi k / n)
    float* sx = reinterpret_cast<float*>(host.data() + t.sx);
    for (int k = 0; k <= L; ++k) {
      double s = std::sin(M_PI * (double)k / (2.0 * L));
      sx[k] = (float)(4.0 * s * s);
    }
    float* sy = reinterpret_cast<float*>(host.data() + t.sy);
    for (int l = 0; l < L; ++l) {
      double s = std::sin(M_PI * (double)l / (double)L);
      sy[l] = (float)(4.0 * s * s);
    }
    // the row transforms' twiddles as a P x (Q|1) matrix, entry [k1][t] =
    // exp(-2 pi i t k1 / L): lanes that walk either index hit distinct banks
    const LenOps* o = kOps[i]();
    const int P = o->P, Q = o->Q, QP = Q | 1;
    t.twm = put(sizeof(cf) * P * QP);
    cf* twm = reinterpret_cast<cf*>(host.data() + t.twm);
    tw = reinterpret_cast<cf*>(host.data() + t.tw);
    for (int k1 = 0; k1 < P; ++k1)
      for (int q = 0; q < QP; ++q) twm[k1 * QP + q] = q < Q ? tw[q * k1] : cf{0.0f, 0.0f};
    tab[L] = t;
  }
  // lengths of the runtime-length passes: the same vectors, no matrix
  for (int L = 2; L <= kMaxGenericLen; ++L) {
    if (!generic_length(L)) continue;
    LenTables t;
    t.tw = put(sizeof(cf) * L);
    t.tw2 = put(sizeof(cf) * (L + 1));
    t.sx = put(sizeof(float) * (L + 1));
    t.sy = put(sizeof(float) * L);
    t.twm = t.tw;
    cf* tw = reinterpret_cast<cf*>(host.data() + t.tw);
    for (int j = 0; j < L; ++j) {
      double a = -2.0 * M_PI * (double)j / (double)L;
      tw[j] = cf{(float)std::cos(a), (float)std::sin(a)};
    }
    cf* tw2 = reinterpret_cast<cf*>(host.data() + t.tw2);
    for (int k = 0; k <= L; ++k) {
      double a = -M_PI * (double)k / (double)L;
      tw2[k] = cf{(float)std::cos(a), (float)std::sin(a)};
    }
    float* sx = reinterpret_cast<float*>(host.data() + t.sx);
    for (int k = 0; k <= L; ++k) {
      double sn = std::sin(M_PI * (double)k / (2.0 * L));
      sx[k] = (float)(4.0 * sn * sn);
    }
    float* sy = reinterpret_cast<float*>(host.data() + t.sy);
    for (int l = 0; l < L; ++l) {
      double sn = std::sin(M_PI * (double)l / (double)L);
      sy[l] = (float)(4.0 * sn * sn);
    }
    tab[L] = t;
  }
}

// Single-frame work lists for the three launch shapes of a frame.
static WorkList one_frame(const FrameDesc& d, int items) {
  WorkList wl;
  wl.one = d;
  wl.descs = nullptr;
  wl.starts = nullptr;
  wl.n = 1;
  wl.total = items;
  return wl;
}
static int row_items(const RowVariant* v, int mode, const FrameDesc& d) {
  return d.C * ilsk::row_bands(d, v->rows[mode]);
}
static int col_items(const ColVariant* v, const FrameDesc& d) {
  const int s = v->cols;
  return d.C * ((d.W / 2 + 1 + s - 1) / s);
}

// Elementwise kernels of the luminance mode (ils_apps.hip).
hipError_t ilsk_launch_luma(const float* rgb, float* y, long long plane, hipStream_t st);
hipError_t ilsk_launch_recombine(const float* f, const float* y, const float* v, float* out, long long plane,
                                 hipStream_t st);

hipError_t ilsk_launch_loglum(const float* rgb, float* L, long long plane, float floor_y, hipStream_t st);
hipError_t ilsk_launch_minmax(const float* B, long long plane, float* scratch, float* mm, hipStream_t st);
hipError_t ilsk_launch_tonemap(const float* f, const float* L, const float* B, const float* mm, float log_contrast,
                               float detail, float* out, long long plane, hipStream_t st);
hipError_t ilsk_launch_tonemap_ms(const float* f, const float* L, const float* const* B, const float* w, int K,
                                  const float* mm, float log_contrast, float* out, long long plane, hipStream_t st);

// ---------------------------------------------------------------- tuner
// Lengths of 480 and more offer two row-band and two column-tile shapes.
// The first call for an image size times each shape on the plan's stream
// (HIP events, a few launches on workspace data, so it synchronises once)
// and keeps the faster; the choice does not change any result bit, since
// every row and column goes through the same arithmetic in either shape.
// ILS_TUNE=0 keeps the default shapes; ILS_TUNE_CACHE names a text file of
// earlier choices ("arch H W C row col" per line) that is read at plan
// creation and appended to.
struct Pick {
  const RowVariant* rv;
  const ColVariant* cv;
};

// H and W stay below 2^16 (compiled lengths); C counts every channel of a
// batch class.
static long long size_key(int H, int W, int C) {
  return ((long long)H << 48) | ((long long)W << 32) | (long long)(unsigned)C;
}

static void load_tune_cache(ils_plan* plan) {
  const char* path = std::getenv("ILS_TUNE_CACHE");
  if (!path) return;
  FILE* fh = std::fopen(path, "r");
  if (!fh) return;
  char arch[64];
  int H, W, C, g, sc;
  while (std::fscanf(fh, "%63s %d %d %d %d %d", arch, &H, &W, &C, &g, &sc) == 6) {
    if (plan->arch != arch || !find_ops(H) || W < 2 || (W & 1) || !find_ops(W / 2)) continue;
    const LenOps* orow = find_ops(W / 2);
    const LenOps* ocol = find_ops(H);
    int r = -1, c = -1;
    for (int i = 0; i < orow->nrow; ++i)
      if (orow->row[i].rows[ilsk::ROW_MID] == g) r = i;
    for (int i = 0; i < ocol->ncol; ++i)
      if (ocol->col[i].cols == sc) c = i;
    if (r >= 0 && c >= 0) plan->tuned[size_key(H, W, C)] = {r, c};
  }
  std::fclose(fh);
}

static float time_launches(ils_plan* plan, const std::function<hipError_t()>& launch) {
  hipEvent_t a = nullptr, b = nullptr;
  float best = 1e30f;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) best = -1.0f;
  for (int rep = 0; rep < 4 && best >= 0.0f; ++rep) {
    float ms = 0.0f;
    if (launch() != hipSuccess || hipEventRecord(a, plan->stream) != hipSuccess || launch() != hipSuccess ||
        launch() != hipSuccess || hipEventRecord(b, plan->stream) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
        hipEventElapsedTime(&ms, a, b) != hipSuccess) {
      best = -1.0f;
      break;
    }
    best = ms < best ? ms : best;
  }
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  return best;
}

// A frame with a row or column length that has no compiled split runs
// every pass on the runtime-length kernels.
static bool frame_generic(int H, int W) { return !find_ops(W / 2) || !find_ops(H); }

// Row bands of a single frame on `cus` compute units with row shape v: the
// fewest rounds of resident blocks that the shape's full bands need, filled
// with as many (shorter, balanced) bands as they hold, but bands of at least
// four rows (or the shape's height, if less).  The blocks of a round then
// end together instead of the last round running a few blocks alone.  Two
// blocks of a shape count as resident on one CU when its LDS allows it and
// a block has at most four waves (one wave of each per SIMD).  The
// runtime-length kernels keep their own bands.
static FrameDesc banded(int cus, const RowVariant* v, FrameDesc d) {
  d.nb_row = 0;
  if (cus <= 0 || frame_generic(d.H, d.W)) return d;
  const int g = v->rows[ilsk::ROW_MID];
  const int lo = (d.H + g - 1) / g;
  const int per_cu = (v->threads + 63) / 64 <= 4 ? ilsk::resident_blocks(v->lds_bytes) : 1;
  const long long per_round = (long long)cus * per_cu;
  const long long rounds = ((long long)d.C * lo + per_round - 1) / per_round;
  const int hi = std::max(lo, d.H / std::min(g, 4));
  d.nb_row = (int)std::max<long long>(lo, std::min<long long>(rounds * per_round / d.C, hi));
  return d;
}

// Default shapes (no tuning).
static Pick default_pick(int H, int W) {
  if (frame_generic(H, W)) {
    const LenOps* g = ilsk_generic_ops(H);
    return Pick{&g->row[0], &g->col[0]};
  }
  return Pick{&find_ops(W / 2)->row[0], &find_ops(H)->col[0]};
}

static Pick choose(ils_plan* plan, const FrameDesc& d) {
  if (frame_generic(d.H, d.W)) return default_pick(d.H, d.W);
  const LenOps* orow = find_ops(d.W / 2);
  const LenOps* ocol = find_ops(d.H);
  Pick pk{&orow->row[0], &ocol->col[0]};
  if (orow->nrow < 2 && ocol->ncol < 2) return pk;
  const long long key = size_key(d.H, d.W, d.C);
  auto it = plan->tuned.find(key);
  if (it == plan->tuned.end()) {
    std::pair<int, int> ch{0, 0};
    const char* env = std::getenv("ILS_TUNE");
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    const bool capturing = hipStreamIsCapturing(plan->stream, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone;
    // a stream under capture cannot be timed, and timing launches would
    // disturb pass profiling: such a call keeps the defaults and leaves the
    // size untuned
    if (capturing || plan->prof_on) return pk;
    if (!(env && std::strcmp(env, "0") == 0)) {
      // time the shapes on the workspace (inputs and outputs point at the
      // second half spectrum: any finite or non-finite data times the same)
      FrameDesc t = d;
      t.f = t.u0 = reinterpret_cast<const float*>(t.specB);
      t.out = reinterpret_cast<float*>(t.specB);
      float bestr = 1e30f, bestc = 1e30f;
      for (int v = 0; v < orow->nrow; ++v) {
        const FrameDesc tb = banded(plan->cus, &orow->row[v], t);
        const WorkList wl = one_frame(tb, row_items(&orow->row[v], ilsk::ROW_MID, tb));
        const float ms = time_launches(plan, [&] { return orow->row[v].launch(ilsk::ROW_MID, ilsk::PEN_CHARBONNIER, wl, plan->stream); });
        if (ms >= 0.0f && ms < bestr) {
          bestr = ms;
          ch.first = v;
        }
      }
      for (int v = 0; v < ocol->ncol; ++v) {
        const WorkList wl = one_frame(t, col_items(&ocol->col[v], t));
        const float ms = time_launches(plan, [&] { return ocol->col[v].launch(wl, plan->stream); });
        if (ms >= 0.0f && ms < bestc) {
          bestc = ms;
          ch.second = v;
        }
      }
      const char* path = std::getenv("ILS_TUNE_CACHE");
      if (path) {
        FILE* fh = std::fopen(path, "a");
        if (fh) {
          std::fprintf(fh, "%s %d %d %d %d %d\n", plan->arch.c_str(), d.H, d.W, d.C,
                       orow->row[ch.first].rows[ilsk::ROW_MID], ocol->col[ch.second].cols);
          std::fclose(fh);
        }
      }
    }
    it = plan->tuned.emplace(key, ch).first;
  }
  pk.rv = &orow->row[it->second.first < orow->nrow ? it->second.first : 0];
  pk.cv = &ocol->col[it->second.second < ocol->ncol ? it->second.second : 0];
  return pk;
}

// Enqueue Algorithm 1 for one frame (N >= 1, lambda > 0): one block per
// work item, 2N + 1 launches.
// The 2N + 1 launches of one frame with the given shapes on stream st;
// wrap(kind, launch) issues each launch (kind as in ils_profile_end).
template <class Wrap>
static hipError_t enqueue_frame(const Pick& pk, const FrameDesc& d0, int N, int pen, int cus, hipStream_t st,
                                Wrap&& wrap) {
  const FrameDesc d = banded(cus, pk.rv, d0);
  const WorkList wrow = one_frame(d, row_items(pk.rv, ilsk::ROW_MID, d));
  const WorkList wfin = one_frame(d, row_items(pk.rv, ilsk::ROW_FINAL, d));
  const WorkList wcol = one_frame(d, col_items(pk.cv, d));
  const int first = (d.f == d.u0) ? ilsk::ROW_FIRST_SAME : ilsk::ROW_FIRST;
  hipError_t e = wrap(0, [&] { return pk.rv->launch(first, pen, wrow, st); });
  for (int n = 0; n < N && e == hipSuccess; ++n) {
    e = wrap(3, [&] { return pk.cv->launch(wcol, st); });
    if (e != hipSuccess) break;
    if (n + 1 < N)
      e = wrap(1, [&] { return pk.rv->launch(ilsk::ROW_MID, pen, wrow, st); });
    else
      e = wrap(2, [&] { return pk.rv->launch(ilsk::ROW_FINAL, pen, wfin, st); });
  }
  return e;
}

// The persistent single-launch sequence for frames of d's size with N iterations
// and `channels` channels in all, or nullptr (none compiled for the size,
// switched off, pass timing active, or its control block would not fit).
static const ilsk::PersistOps* persist_for(const ils_plan* plan, const FrameDesc& d, int N, long long channels) {
  if (!plan->persist_on || plan->prof_on || N < 1) return nullptr;
  if (ilsk::kPersistCtlHead + (2LL * N + 1) * channels > (long long)kPersistCtlInts) return nullptr;
  return find_persist(d.W / 2, d.H);
}

// Enqueue one persistent launch: frames from the device descriptor array descs
// (channel prefix sums ch_start), or the single frame `one` when descs is
// null; control block at ctl (ctl_ints ints) in the workspace header.
static hipError_t enqueue_persist(ils_plan* plan, const ilsk::PersistOps* fo, const FrameDesc* descs,
                                const int* ch_start, const FrameDesc& one, int n, int C, long long channels, int N,
                                int pen, int first, int* ctl, hipStream_t st) {
  if (plan->cus <= 0) {
    hipDeviceProp_t prop;
    hipError_t e = hipGetDeviceProperties(&prop, plan->device);
    if (e != hipSuccess) return e;
    plan->cus = prop.multiProcessorCount;
  }
  const int per_cu = fo->per_cu(pen);
  if (per_cu <= 0) return hipErrorInvalidConfiguration;
  ilsk::PersistList fl;
  fl.descs = descs;
  fl.one = one;
  fl.ctl = ctl;
  fl.err = reinterpret_cast<int*>(plan->ws + kPersistErrOff);
  fl.ch_start = ch_start;
  fl.n = n;
  fl.C = C;
  fl.N = N;
  fl.first = first;
  fl.nb_row = (one.H + fo->rows - 1) / fo->rows;
  fl.nb_col = (one.W / 2 + 1 + fo->cols - 1) / fo->cols;
  fl.wait_ticks = plan->wait_ticks;
  const long long items = channels * ((N + 1LL) * fl.nb_row + (long long)N * fl.nb_col);
  const long long grid = std::min<long long>(items, (long long)per_cu * plan->cus);
  const int ctl_ints = (int)(ilsk::kPersistCtlHead + (2LL * N + 1) * channels);
  return fo->launch(pen, fl, ctl_ints, (int)grid, st);
}

static int run_frame(ils_plan* plan, const FrameDesc& d, int N, int pen = ilsk::PEN_CHARBONNIER) {
  if (const ilsk::PersistOps* fo = persist_for(plan, d, N, d.C)) {
    const int first = (d.f == d.u0) ? ilsk::ROW_FIRST_SAME : ilsk::ROW_FIRST;
    int* ctl = reinterpret_cast<int*>(plan->ws + kBatchListBytes);
    return record(plan, enqueue_persist(plan, fo, nullptr, nullptr, d, 1, d.C, d.C, N, pen, first, ctl, plan->stream));
  }
  const Pick pk = choose(plan, d);
  const hipError_t e = enqueue_frame(pk, d, N, pen, plan->cus, plan->stream, [&](int kind, auto&& launch) {
    return timed(plan, kind, launch);
  });
  return record(plan, e);
}

// --------------------------------------------------------------- C ABI
extern "C" {

const char* ils_status_string(int status) {
  switch (status) {
    case ILS_OK: return "ok";
    case ILS_ERR_INVALID_ARG: return "invalid argument";
    case ILS_ERR_UNSUPPORTED_SIZE: return "unsupported image size";
    case ILS_ERR_WORKSPACE: return "workspace missing or too small";
    case ILS_ERR_HIP: return "HIP runtime error";
    case ILS_ERR_NOT_CALIBRATED: return "surrogate gate not calibrated";
    default: return "unknown status";
  }
}

int ils_length_supported(int L) { return (find_ops(L) != nullptr || generic_length(L)) ? 1 : 0; }

int ils_size_supported(int H, int W) {
  if (H < 2 || W < 2 || (W & 1)) return 0;
  return ils_length_supported(H) && ils_length_supported(W / 2);
}

int ils_check_args(int H, int W, int C, float lambda, float p, float eps, int N) {
  int rc = check_params(lambda, p, eps, N);
  if (rc != ILS_OK) return rc;
  return check_size(nullptr, H, W, C);
}

size_t ils_workspace_bytes(int max_H, int max_W, int max_C, int max_frames) {
  if (max_H < 2 || max_W < 2 || max_C < 1 || max_frames < 1) return 0;
  return kBatchHeaderBytes + (size_t)max_frames * frame_ws_bytes(max_H, max_W, max_C);
}

size_t ils_batch_workspace_bytes(const ils_frame* frames, int n) {
  if (!frames || n < 1) return 0;
  size_t s = kBatchHeaderBytes;
  for (int i = 0; i < n; ++i) {
    if (frames[i].H < 2 || frames[i].W < 2 || frames[i].C < 1) return 0;
    s += frame_ws_bytes(frames[i].H, frames[i].W, frames[i].C);
  }
  return s;
}

int ils_plan_create(ils_plan** plan_out, int max_H, int max_W, int max_C, int max_frames,
                    void* workspace, size_t ws_bytes, void* hip_stream, unsigned flags) {
  if (!plan_out) return ILS_ERR_INVALID_ARG;
  *plan_out = nullptr;
  if (max_H < 2 || max_W < 2 || max_C < 1 || max_frames < 1) return ILS_ERR_INVALID_ARG;
  if (flags & ~(unsigned)ILS_PLAN_NO_GRAPH) return ILS_ERR_INVALID_ARG;
  if (!workspace || ((uintptr_t)workspace & 255)) return ILS_ERR_WORKSPACE;
  // room for one frame of the largest size; batched calls check their exact need
  if (ws_bytes < ils_workspace_bytes(max_H, max_W, max_C, 1)) return ILS_ERR_WORKSPACE;

  ils_plan* plan = new (std::nothrow) ils_plan();
  if (!plan) return ILS_ERR_HIP;
  plan->max_H = max_H;
  plan->max_W = max_W;
  plan->max_C = max_C;
  plan->max_frames = max_frames;
  plan->ws = static_cast<char*>(workspace);
  plan->ws_bytes = ws_bytes;
  plan->stream = static_cast<hipStream_t>(hip_stream);
  plan->flags = flags;
  plan->last_error = ILS_OK;
  plan->tables = nullptr;
  plan->stage_next = 0;
  plan->prof_on = false;
  plan->persist_on = false;  // switched off: see ils_plan_set_persistent
  plan->cus = 0;
  plan->wait_ticks = kPersistWaitTicks;
  plan->ev_used = 0;
  plan->cap_stream = nullptr;
  for (int c = 0; c < kChains; ++c) {
    plan->chain_stream[c] = nullptr;
    plan->join_ev[c] = nullptr;
  }
  plan->fork_ev = nullptr;
  for (int i = 0; i < kStageSlots; ++i) {
    plan->stage[i] = nullptr;
    plan->stage_ev[i] = nullptr;
    plan->stage_used[i] = false;
  }
  if (hipGetDevice(&plan->device) != hipSuccess) {
    delete plan;
    return ILS_ERR_HIP;
  }
  {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, plan->device) == hipSuccess) {
      plan->arch = prop.gcnArchName;
      plan->cus = prop.multiProcessorCount;
    }
    const size_t colon = plan->arch.find(':');
    if (colon != std::string::npos) plan->arch.resize(colon);
    load_tune_cache(plan);
  }
  if (!(flags & ILS_PLAN_NO_GRAPH)) {
    bool ok = hipStreamCreateWithFlags(&plan->cap_stream, hipStreamNonBlocking) == hipSuccess &&
              hipEventCreateWithFlags(&plan->fork_ev, hipEventDisableTiming) == hipSuccess;
    for (int c = 1; c < kChains && ok; ++c)
      ok = hipStreamCreateWithFlags(&plan->chain_stream[c], hipStreamNonBlocking) == hipSuccess &&
           hipEventCreateWithFlags(&plan->join_ev[c], hipEventDisableTiming) == hipSuccess;
    if (!ok) {
      free_plan(plan);
      return ILS_ERR_HIP;
    }
    plan->chain_stream[0] = plan->cap_stream;
  }
  for (int i = 0; i < kStageSlots; ++i) {
    if (hipHostMalloc((void**)&plan->stage[i], kStageBytes, hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&plan->stage_ev[i], hipEventDisableTiming) != hipSuccess) {
      free_plan(plan);
      return ILS_ERR_HIP;
    }
  }

  std::vector<char> host;
  build_tables(host, plan->tab);
  hipError_t e = hipMalloc(&plan->tables, host.size());
  if (e == hipSuccess) e = hipMemcpy(plan->tables, host.data(), host.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(plan->ws + kPersistErrOff, 0, sizeof(int));
  if (e != hipSuccess) {
    free_plan(plan);
    return ILS_ERR_HIP;
  }
  *plan_out = plan;
  return ILS_OK;
}

int ils_plan_set_persistent(ils_plan* plan, int on) {
  if (!plan || (on != 0 && on != 1)) return ILS_ERR_INVALID_ARG;
  // The persistent launch is switched off: its first launches did not end
  // on the GPU, for a reason not found yet.  Only "off" is accepted.
  if (on) return ILS_ERR_INVALID_ARG;
  plan->persist_on = false;
  return ILS_OK;
}

int ils_plan_set_wait_limit(ils_plan* plan, long long microseconds) {
  if (!plan || microseconds < 0) return ILS_ERR_INVALID_ARG;
  plan->wait_ticks = microseconds == 0 ? kPersistWaitTicks : microseconds * 100;
  return ILS_OK;
}

int ils_plan_set_stream(ils_plan* plan, void* hip_stream) {
  if (!plan) return ILS_ERR_INVALID_ARG;
  plan->stream = static_cast<hipStream_t>(hip_stream);
  return ILS_OK;
}

int ils_plan_destroy(ils_plan* plan) {
  if (!plan) return ILS_OK;
  free_plan(plan);
  return ILS_OK;
}

int ils_profile_begin(ils_plan* plan) {
  if (!plan) return ILS_ERR_INVALID_ARG;
  plan->prof_on = true;
  plan->ev_used = 0;
  plan->prof_kind.clear();
  return ILS_OK;
}

int ils_profile_end(ils_plan* plan, double* total_ms, int* count) {
  if (!plan || !total_ms || !count) return ILS_ERR_INVALID_ARG;
  plan->prof_on = false;
  for (int k = 0; k < 4; ++k) {
    total_ms[k] = 0.0;
    count[k] = 0;
  }
  if (plan->ev_used == 0) return ILS_OK;
  hipError_t e = hipEventSynchronize(plan->ev_pool[plan->ev_used - 1]);
  if (e != hipSuccess) return record(plan, e);
  for (size_t i = 0; i < plan->prof_kind.size(); ++i) {
    float ms = 0.0f;
    e = hipEventElapsedTime(&ms, plan->ev_pool[2 * i], plan->ev_pool[2 * i + 1]);
    if (e != hipSuccess) return record(plan, e);
    total_ms[plan->prof_kind[i]] += ms;
    count[plan->prof_kind[i]] += 1;
  }
  plan->ev_used = 0;
  plan->prof_kind.clear();
  return ILS_OK;
}

int ils_last_error(ils_plan* plan) {
  if (!plan) return ILS_ERR_INVALID_ARG;
  hipError_t e = hipStreamQuery(plan->stream);
  if (e != hipSuccess && e != hipErrorNotReady) record(plan, e);
  if (e == hipSuccess) {  // stream idle: read and clear the persistent launches' wait-expiry word
    int word = 0;
    if (hipMemcpy(&word, plan->ws + kPersistErrOff, sizeof(int), hipMemcpyDeviceToHost) == hipSuccess && word != 0) {
      (void)hipMemset(plan->ws + kPersistErrOff, 0, sizeof(int));
      if (plan->last_error == ILS_OK) plan->last_error = ILS_ERR_HIP;
    }
  }
  int r = plan->last_error;
  plan->last_error = ILS_OK;
  return r;
}

int ils_shape_variants(int H, int W, int* n_row, int* n_col) {
  if (!n_row || !n_col) return ILS_ERR_INVALID_ARG;
  if (!ils_size_supported(H, W)) return ILS_ERR_UNSUPPORTED_SIZE;
  if (frame_generic(H, W)) {
    *n_row = *n_col = 1;
    return ILS_OK;
  }
  *n_row = find_ops(W / 2)->nrow;
  *n_col = find_ops(H)->ncol;
  return ILS_OK;
}

int ils_plan_tune(ils_plan* plan, int H, int W, int C, int* row_shape, int* col_shape) {
  if (!plan || !row_shape || !col_shape) return ILS_ERR_INVALID_ARG;
  const int rc = check_size(plan, H, W, C);
  if (rc != ILS_OK) return rc;
  FrameDesc d;
  fill_desc(plan, d, H, W, C, 1.0f, 1.0f, 1e-4f);
  char* base = plan->ws + kBatchHeaderBytes;
  d.specA = reinterpret_cast<cf*>(base);
  d.specB = reinterpret_cast<cf*>(base + (size_t)C * H * d.ldS * sizeof(cf));
  d.f = d.u0 = reinterpret_cast<const float*>(d.specB);
  d.out = reinterpret_cast<float*>(d.specB);
  const Pick pk = choose(plan, d);
  if (frame_generic(H, W)) {
    *row_shape = *col_shape = 0;
    return ILS_OK;
  }
  *row_shape = (int)(pk.rv - find_ops(W / 2)->row);
  *col_shape = (int)(pk.cv - find_ops(H)->col);
  return ILS_OK;
}

int ils_plan_set_shapes(ils_plan* plan, int H, int W, int C, int row_shape, int col_shape) {
  if (!plan) return ILS_ERR_INVALID_ARG;
  const int rc = check_size(plan, H, W, C);
  if (rc != ILS_OK) return rc;
  int nr = 1, nc = 1;
  (void)ils_shape_variants(H, W, &nr, &nc);
  if (row_shape < 0 || row_shape >= nr || col_shape < 0 || col_shape >= nc) return ILS_ERR_INVALID_ARG;
  if (frame_generic(H, W)) return ILS_OK;
  plan->tuned[size_key(H, W, C)] = {row_shape, col_shape};
  return ILS_OK;
}

int ils_iterate_from(ils_plan* plan, const float* f, const float* u0, int H, int W, int C,
                     float lambda, float p, float eps, int N, float* out) {
  if (!plan || !f || !u0 || !out) return ILS_ERR_INVALID_ARG;
  int rc = check_params(lambda, p, eps, N);
  if (rc != ILS_OK) return rc;
  rc = check_size(plan, H, W, C);
  if (rc != ILS_OK) return rc;
  const size_t need = frame_ws_bytes(H, W, C);
  if (plan->ws_bytes < kBatchHeaderBytes + need) return ILS_ERR_WORKSPACE;
  const size_t img = (size_t)C * H * W * sizeof(float);
  if (N == 0 || lambda == 0.0f) {
    // u^N = u0 for N = 0; for lambda = 0 the LS problem gives u = f.
    const float* src = (N == 0) ? u0 : f;
    if (src == out) return ILS_OK;
    return record(plan, hipMemcpyAsync(out, src, img, hipMemcpyDeviceToDevice, plan->stream));
  }
  FrameDesc d;
  fill_desc(plan, d, H, W, C, lambda, p, eps);
  d.f = f;
  d.u0 = u0;
  d.out = out;
  char* base = plan->ws + kBatchHeaderBytes;
  const size_t half = (size_t)C * H * d.ldS * sizeof(cf);
  d.specA = reinterpret_cast<cf*>(base);
  d.specB = reinterpret_cast<cf*>(base + half);
  return run_frame(plan, d, N);
}

int ils_iterate_from_c(ils_plan* plan, const float* f, const float* u0, int H, int W, int C, float lambda,
                       float p, float eps, float c, int N, float* out) {
  if (!plan || !f || !u0 || !out) return ILS_ERR_INVALID_ARG;
  int rc = check_params(lambda, p, eps, N);
  if (rc != ILS_OK) return rc;
  const double c0 = (double)p * std::pow((double)eps, (double)p / 2.0 - 1.0);  // Eq. (11)
  if (!finite_f(c) || (double)c < c0 * (1.0 - 1e-6)) return ILS_ERR_INVALID_ARG;
  rc = check_size(plan, H, W, C);
  if (rc != ILS_OK) return rc;
  const size_t need = frame_ws_bytes(H, W, C);
  if (plan->ws_bytes < kBatchHeaderBytes + need) return ILS_ERR_WORKSPACE;
  if (N == 0 || lambda == 0.0f) {
    const float* src = (N == 0) ? u0 : f;
    if (src == out) return ILS_OK;
    return record(plan, hipMemcpyAsync(out, src, (size_t)C * H * W * sizeof(float), hipMemcpyDeviceToDevice,
                                       plan->stream));
  }
  FrameDesc d;
  fill_desc(plan, d, H, W, C, lambda, p, eps);
  // c within float rounding of c0 is c0 itself (the default path, bit for bit)
  if (std::fabs((double)c - c0) > 1e-6 * c0) {
    d.kappa = (float)((double)lambda * (double)c / 2.0);
    d.log2_r = (float)std::log2(c0 / (double)c);
  }
  d.f = f;
  d.u0 = u0;
  d.out = out;
  char* base = plan->ws + kBatchHeaderBytes;
  d.specA = reinterpret_cast<cf*>(base);
  d.specB = reinterpret_cast<cf*>(base + (size_t)C * H * d.ldS * sizeof(cf));
  return run_frame(plan, d, N);
}

int ils_smooth(ils_plan* plan, const float* f, int H, int W, int C, float lambda, float p,
               float eps, int N, float* out) {
  return ils_iterate_from(plan, f, f, H, W, C, lambda, p, eps, N, out);
}

int ils_smooth_welsch(ils_plan* plan, const float* f, int H, int W, int C, float lambda, float gamma,
                      int N, float* out) {
  if (!plan || !f || !out) return ILS_ERR_INVALID_ARG;
  int rc = check_params_welsch(lambda, gamma, N);
  if (rc != ILS_OK) return rc;
  rc = check_size(plan, H, W, C);
  if (rc != ILS_OK) return rc;
  const size_t need = frame_ws_bytes(H, W, C);
  if (plan->ws_bytes < kBatchHeaderBytes + need) return ILS_ERR_WORKSPACE;
  if (N == 0 || lambda == 0.0f) {
    if (f == out) return ILS_OK;
    return record(plan, hipMemcpyAsync(out, f, (size_t)C * H * W * sizeof(float), hipMemcpyDeviceToDevice,
                                       plan->stream));
  }
  FrameDesc d;
  fill_desc_welsch(plan, d, H, W, C, lambda, gamma);
  d.f = f;
  d.u0 = f;
  d.out = out;
  char* base = plan->ws + kBatchHeaderBytes;
  d.specA = reinterpret_cast<cf*>(base);
  d.specB = reinterpret_cast<cf*>(base + (size_t)C * H * d.ldS * sizeof(cf));
  return run_frame(plan, d, N, ilsk::PEN_WELSCH);
}

int ils_detail_enhance(ils_plan* plan, const float* f, int H, int W, int C, float lambda, float p, float eps,
                       int N, float k, float* out) {
  if (!plan || !f || !out || !finite_f(k)) return ILS_ERR_INVALID_ARG;
  int rc = check_params(lambda, p, eps, N);
  if (rc != ILS_OK) return rc;
  rc = check_size(plan, H, W, C);
  if (rc != ILS_OK) return rc;
  const size_t need = frame_ws_bytes(H, W, C);
  if (plan->ws_bytes < kBatchHeaderBytes + need) return ILS_ERR_WORKSPACE;
  if (N == 0 || lambda == 0.0f) {  // u = f, so u + k (f - u) = f
    if (f == out) return ILS_OK;
    return record(plan, hipMemcpyAsync(out, f, (size_t)C * H * W * sizeof(float), hipMemcpyDeviceToDevice,
                                       plan->stream));
  }
  FrameDesc d;
  fill_desc(plan, d, H, W, C, lambda, p, eps);
  d.f = f;
  d.u0 = f;
  d.out = out;
  d.boost = k;
  char* base = plan->ws + kBatchHeaderBytes;
  d.specA = reinterpret_cast<cf*>(base);
  d.specB = reinterpret_cast<cf*>(base + (size_t)C * H * d.ldS * sizeof(cf));
  return run_frame(plan, d, N);
}

size_t ils_luminance_workspace_bytes(int max_H, int max_W) {
  if (max_H < 2 || max_W < 2 || (max_W & 1)) return 0;
  return kBatchHeaderBytes + frame_ws_bytes(max_H, max_W, 1) + 2 * align_up((size_t)max_H * max_W * sizeof(float), 256);
}

int ils_smooth_luminance(ils_plan* plan, const float* f, int H, int W, float lambda, float p, float eps, int N,
                         float k, float* out) {
  if (!plan || !f || !out || !finite_f(k)) return ILS_ERR_INVALID_ARG;
  int rc = check_params(lambda, p, eps, N);
  if (rc != ILS_OK) return rc;
  rc = check_size(plan, H, W, 1);
  if (rc != ILS_OK) return rc;
  if (plan->ws_bytes < ils_luminance_workspace_bytes(H, W)) return ILS_ERR_WORKSPACE;
  const long long plane = (long long)H * W;
  char* base = plan->ws + kBatchHeaderBytes;
  const size_t spec = frame_ws_bytes(H, W, 1);
  float* Y = reinterpret_cast<float*>(base + spec);
  float* V = reinterpret_cast<float*>(base + spec + align_up((size_t)plane * sizeof(float), 256));
  hipError_t e = ilsk_launch_luma(f, Y, plane, plan->stream);
  if (e != hipSuccess) return record(plan, e);
  if (N == 0 || lambda == 0.0f) {  // u = Y: the output is the input
    if (f == out) return ILS_OK;
    return record(plan, hipMemcpyAsync(out, f, 3 * (size_t)plane * sizeof(float), hipMemcpyDeviceToDevice,
                                       plan->stream));
  }
  FrameDesc d;
  fill_desc(plan, d, H, W, 1, lambda, p, eps);
  d.f = Y;
  d.u0 = Y;
  d.out = V;
  d.boost = k;  // V = u + k (Y - u)
  d.specA = reinterpret_cast<cf*>(base);
  d.specB = reinterpret_cast<cf*>(base + (size_t)H * d.ldS * sizeof(cf));
  rc = run_frame(plan, d, N);
  if (rc != ILS_OK) return rc;
  return record(plan, ilsk_launch_recombine(f, Y, V, out, plane, plan->stream));
}

int ils_tone_map(ils_plan* plan, const float* f, int H, int W, float lambda, float p, float eps, int N,
                 float contrast, float detail, float* out) {
  if (!plan || !f || !out || !finite_f(contrast) || !(contrast > 1.0f) || !finite_f(detail) || detail < 0.0f)
    return ILS_ERR_INVALID_ARG;
  int rc = check_params(lambda, p, eps, N);
  if (rc != ILS_OK) return rc;
  rc = check_size(plan, H, W, 1);
  if (rc != ILS_OK) return rc;
  if (plan->ws_bytes < ils_luminance_workspace_bytes(H, W)) return ILS_ERR_WORKSPACE;
  const long long plane = (long long)H * W;
  char* base = plan->ws + kBatchHeaderBytes;
  const size_t spec = frame_ws_bytes(H, W, 1);
  float* L = reinterpret_cast<float*>(base + spec);
  float* B = reinterpret_cast<float*>(base + spec + align_up((size_t)plane * sizeof(float), 256));
  float* scratch = reinterpret_cast<float*>(plan->ws);  // header: min/max partials, then the pair
  float* mm = scratch + 2 * 256;
  hipError_t e = ilsk_launch_loglum(f, L, plane, 1e-6f, plan->stream);
  if (e != hipSuccess) return record(plan, e);
  if (N == 0 || lambda == 0.0f) {
    e = hipMemcpyAsync(B, L, (size_t)plane * sizeof(float), hipMemcpyDeviceToDevice, plan->stream);
    if (e != hipSuccess) return record(plan, e);
  } else {
    FrameDesc d;
    fill_desc(plan, d, H, W, 1, lambda, p, eps);
    d.f = L;
    d.u0 = L;
    d.out = B;
    d.specA = reinterpret_cast<cf*>(base);
    d.specB = reinterpret_cast<cf*>(base + (size_t)H * d.ldS * sizeof(cf));
    rc = run_frame(plan, d, N);
    if (rc != ILS_OK) return rc;
  }
  e = ilsk_launch_minmax(B, plane, scratch, mm, plan->stream);
  if (e == hipSuccess)
    e = ilsk_launch_tonemap(f, L, B, mm, (float)std::log((double)contrast), detail, out, plane, plan->stream);
  return record(plan, e);
}

size_t ils_tone_map_multiscale_workspace_bytes(int max_H, int max_W, int K) {
  if (max_H < 2 || max_W < 2 || (max_W & 1) || K < 1 || K > ILS_MAX_SCALES) return 0;
  return kBatchHeaderBytes + frame_ws_bytes(max_H, max_W, 1) +
         (size_t)(K + 1) * align_up((size_t)max_H * max_W * sizeof(float), 256);
}

int ils_tone_map_multiscale(ils_plan* plan, const float* f, int H, int W, const float* lambdas,
                            const float* weights, int K, float p, float eps, int N, float contrast, float* out) {
  if (!plan || !f || !out || !lambdas || !weights || K < 1 || K > ILS_MAX_SCALES) return ILS_ERR_INVALID_ARG;
  if (!finite_f(contrast) || !(contrast > 1.0f)) return ILS_ERR_INVALID_ARG;
  for (int k = 0; k < K; ++k) {
    if (!finite_f(weights[k]) || weights[k] < 0.0f) return ILS_ERR_INVALID_ARG;
    int rc = check_params(lambdas[k], p, eps, N);
    if (rc != ILS_OK) return rc;
  }
  int rc = check_size(plan, H, W, 1);
  if (rc != ILS_OK) return rc;
  if (plan->ws_bytes < ils_tone_map_multiscale_workspace_bytes(H, W, K)) return ILS_ERR_WORKSPACE;
  const long long plane = (long long)H * W;
  const size_t plane_b = align_up((size_t)plane * sizeof(float), 256);
  char* base = plan->ws + kBatchHeaderBytes;
  const size_t spec = frame_ws_bytes(H, W, 1);
  float* L = reinterpret_cast<float*>(base + spec);
  const float* B[ILS_MAX_SCALES];
  float* scratch = reinterpret_cast<float*>(plan->ws);  // header: min/max partials, then the pair
  float* mm = scratch + 2 * 256;
  hipError_t e = ilsk_launch_loglum(f, L, plane, 1e-6f, plan->stream);
  if (e != hipSuccess) return record(plan, e);
  // every level is smoothed from L itself (not from the previous level)
  for (int k = 0; k < K; ++k) {
    float* Bk = reinterpret_cast<float*>(base + spec + (size_t)(k + 1) * plane_b);
    B[k] = Bk;
    if (N == 0 || lambdas[k] == 0.0f) {
      e = hipMemcpyAsync(Bk, L, (size_t)plane * sizeof(float), hipMemcpyDeviceToDevice, plan->stream);
      if (e != hipSuccess) return record(plan, e);
      continue;
    }
    FrameDesc d;
    fill_desc(plan, d, H, W, 1, lambdas[k], p, eps);
    d.f = L;
    d.u0 = L;
    d.out = Bk;
    d.specA = reinterpret_cast<cf*>(base);
    d.specB = reinterpret_cast<cf*>(base + (size_t)H * d.ldS * sizeof(cf));
    rc = run_frame(plan, d, N);
    if (rc != ILS_OK) return rc;
  }
  e = ilsk_launch_minmax(B[K - 1], plane, scratch, mm, plan->stream);
  if (e == hipSuccess)
    e = ilsk_launch_tonemap_ms(f, L, B, weights, K, mm, (float)std::log((double)contrast), out, plane, plan->stream);
  return record(plan, e);
}

int ils_smooth_batch(ils_plan* plan, const ils_frame* frames, int n) {
  if (!plan || !frames || n < 1) return ILS_ERR_INVALID_ARG;
  if (n > plan->max_frames || n > kMaxBatchFrames) return ILS_ERR_INVALID_ARG;
  for (int i = 0; i < n; ++i) {
    const ils_frame& fr = frames[i];
    if (!fr.f || !fr.out) return ILS_ERR_INVALID_ARG;
    int rc = check_frame_params(fr);
    if (rc != ILS_OK) return rc;
    rc = check_size(plan, fr.H, fr.W, fr.C);
    if (rc != ILS_OK) return rc;
  }
  const size_t need = ils_batch_workspace_bytes(frames, n);
  if (need == 0 || plan->ws_bytes < need) return ILS_ERR_WORKSPACE;

  // Descriptors for every frame that needs iterations; trivial frames copy.
  std::vector<FrameDesc> descs;
  std::vector<int> iters, pens;
  char* base = plan->ws + kBatchHeaderBytes;
  size_t off = 0;
  for (int i = 0; i < n; ++i) {
    const ils_frame& fr = frames[i];
    const float* u0 = fr.u0 ? fr.u0 : fr.f;
    if (fr.N == 0 || fr.lambda == 0.0f) {
      const float* src = (fr.N == 0) ? u0 : fr.f;
      if (src != fr.out) {
        hipError_t e = hipMemcpyAsync(fr.out, src, (size_t)fr.C * fr.H * fr.W * sizeof(float),
                                      hipMemcpyDeviceToDevice, plan->stream);
        if (e != hipSuccess) return record(plan, e);
      }
      off += frame_ws_bytes(fr.H, fr.W, fr.C);
      continue;
    }
    FrameDesc d;
    if (fr.penalty == ILS_PENALTY_WELSCH)
      fill_desc_welsch(plan, d, fr.H, fr.W, fr.C, fr.lambda, fr.gamma);
    else
      fill_desc(plan, d, fr.H, fr.W, fr.C, fr.lambda, fr.p, fr.eps);
    d.f = fr.f;
    d.u0 = u0;
    d.out = fr.out;
    const size_t half = (size_t)fr.C * fr.H * d.ldS * sizeof(cf);
    d.specA = reinterpret_cast<cf*>(base + off);
    d.specB = reinterpret_cast<cf*>(base + off + half);
    off += frame_ws_bytes(fr.H, fr.W, fr.C);
    descs.push_back(d);
    iters.push_back(fr.N);
    pens.push_back(fr.penalty);
  }
  if (descs.empty()) return ILS_OK;

  // Group frames into classes of equal (row length, column length, N,
  // penalty): one launch per pass per class, each a grid over the class's
  // (frame, channel, band) work list.  A class of frames of one channel
  // count that each hold at least kPartPxCh pixel-channels is cut into one
  // part per frame; any other class into min(frames, kChains) parts of
  // consecutive frames (small frames need the larger grids of a shared
  // launch, and mixed grey and colour frames would make uneven parts).
  // Per-frame parts go to the kChains independent chains in turn, and a
  // chain runs each one's whole pass sequence before the next one's, so the
  // chains drift out of phase and the passes of one run on the compute
  // units the other's leave idle; the parts of any other class go to chains
  // 0, 1, ... and run pass-major, side by side with the other parts of
  // their class.
  struct Class {
    int M, H, N, pen;
    std::vector<int> idx;
    int lane;
    bool big;
  };
  std::vector<Class> grouped;
  for (size_t i = 0; i < descs.size(); ++i) {
    int M = descs[i].W / 2, H = descs[i].H, N = iters[i], pen = pens[i];
    size_t c = 0;
    for (; c < grouped.size(); ++c)
      if (grouped[c].M == M && grouped[c].H == H && grouped[c].N == N && grouped[c].pen == pen) break;
    if (c == grouped.size()) grouped.push_back(Class{M, H, N, pen, {}, 0, false});
    grouped[c].idx.push_back((int)i);
  }
  std::vector<Class> classes;
  int next_big = 0;
  for (const Class& g : grouped) {
    const int nf = (int)g.idx.size();
    bool big = true;
    for (int i : g.idx)
      big = big && (long long)descs[i].C * descs[i].H * descs[i].W >= kPartPxCh && descs[i].C == descs[g.idx[0]].C;
    const int parts = big ? nf : (nf < kChains ? nf : kChains);
    for (int k = 0; k < parts; ++k) {
      Class a = g;
      a.big = big;
      a.idx.assign(g.idx.begin() + (size_t)nf * k / parts, g.idx.begin() + (size_t)nf * (k + 1) / parts);
      if (big) {
        a.lane = next_big;
        next_big = (next_big + 1) % kChains;
      } else {
        a.lane = k;
      }
      classes.push_back(a);
    }
  }

  // Host image of the batch header: per class, descriptors then three start
  // arrays (row FIRST/MID, row FINAL, column).
  std::vector<char> hdr;
  auto put = [&](const void* src, size_t bytes) {
    size_t o = align_up(hdr.size(), 64);
    hdr.resize(o + bytes);
    std::memcpy(hdr.data() + o, src, bytes);
    return o;
  };
  struct Launch {
    Pick pk;
    int N, pen, first, lane;
    bool big;
    WorkList row, fin, col;
    // the part as one persistent launch (fo != nullptr): its frames' channel
    // count (uniform C0, else prefix sums at chs in the header), control block
    const ilsk::PersistOps* fo;
    int C0;
    long long channels;
    const int* chs;
    int* ctl;
    FrameDesc d0;  // the part's first frame (its size)
  };
  std::vector<Launch> launches;
  std::vector<size_t> offs;  // (desc, row starts, fin starts, col starts) per class
  std::vector<long long> chs_offs;  // channel prefix sums of a persistent part with mixed channel counts, or -1
  size_t ctl_used = 0;  // ints of the persistent control area taken
  int nbig = 0;
  for (const Class& cl : classes) nbig += cl.big ? 1 : 0;
  for (const Class& cl : classes) {
    Launch L;
    // shapes are tuned for the class's whole work (all channels of all its
    // frames), timed on a stand-in frame with that many channels laid out
    // over the class's share of the workspace
    FrameDesc tdesc = descs[cl.idx[0]];
    int ctot = 0;
    for (int i : cl.idx) ctot += descs[i].C;
    tdesc.C = ctot;
    tdesc.specA = reinterpret_cast<cf*>(base);
    tdesc.specB = reinterpret_cast<cf*>(base + (size_t)ctot * tdesc.H * tdesc.ldS * sizeof(cf));
    L.pk = choose(plan, tdesc);
    // A per-frame part runs beside the other chain's parts, where the tuner's
    // timing of one launch on an idle chip does not carry over to the column
    // tile: it takes the widest (measured on 32 frames of 4K RGB, N = 10: the
    // four-column tile, fastest alone because two share a CU, made the batch
    // 6 % slower than the eight-column one).
    if (cl.big && nbig >= 2 && !frame_generic(tdesc.H, tdesc.W)) L.pk.cv = &find_ops(tdesc.H)->col[0];
    L.lane = cl.lane;
    L.big = cl.big;
    L.N = cl.N;
    L.pen = cl.pen;
    // the first pass reads the data term as u^0 when every frame of the class has u^0 = f
    L.first = ilsk::ROW_FIRST_SAME;
    for (int i : cl.idx)
      if (descs[i].u0 != descs[i].f) L.first = ilsk::ROW_FIRST;
    std::vector<FrameDesc> cd;
    std::vector<int> srow(1, 0), sfin(1, 0), scol(1, 0);
    for (int i : cl.idx) {
      const FrameDesc& d = descs[i];
      cd.push_back(d);
      const int gr = L.pk.rv->rows[ilsk::ROW_MID], gf = L.pk.rv->rows[ilsk::ROW_FINAL];
      const int sc = L.pk.cv->cols;
      srow.push_back(srow.back() + d.C * ((d.H + gr - 1) / gr));
      sfin.push_back(sfin.back() + d.C * ((d.H + gf - 1) / gf));
      scol.push_back(scol.back() + d.C * ((d.W / 2 + 1 + sc - 1) / sc));
    }
    offs.push_back(put(cd.data(), cd.size() * sizeof(FrameDesc)));
    offs.push_back(put(srow.data(), srow.size() * sizeof(int)));
    offs.push_back(put(sfin.data(), sfin.size() * sizeof(int)));
    offs.push_back(put(scol.data(), scol.size() * sizeof(int)));
    // the part as one persistent launch, when compiled for its size and its
    // control block fits what is left of the control area
    L.fo = persist_for(plan, cd[0], cl.N, ctot);
    L.C0 = cd[0].C;
    L.channels = ctot;
    L.chs = nullptr;
    L.ctl = nullptr;
    L.d0 = cd[0];
    chs_offs.push_back(-1);
    if (L.fo) {
      // whole 128-byte lines, so every ticket counter has a line of its own
      const size_t need_ints = align_up(ilsk::kPersistCtlHead + (2 * (size_t)cl.N + 1) * (size_t)ctot, 32);
      if (ctl_used + need_ints > kPersistCtlInts) {
        L.fo = nullptr;
      } else {
        L.ctl = reinterpret_cast<int*>(plan->ws + kBatchListBytes) + ctl_used;
        ctl_used += need_ints;
        bool uniform = true;
        std::vector<int> chs(1, 0);
        for (const FrameDesc& d : cd) {
          uniform = uniform && d.C == L.C0;
          chs.push_back(chs.back() + d.C);
        }
        if (!uniform) chs_offs.back() = (long long)put(chs.data(), chs.size() * sizeof(int));
      }
    }
    const int nf = (int)cl.idx.size();
    L.row = WorkList{FrameDesc{}, nullptr, nullptr, nf, srow.back()};
    L.fin = WorkList{FrameDesc{}, nullptr, nullptr, nf, sfin.back()};
    L.col = WorkList{FrameDesc{}, nullptr, nullptr, nf, scol.back()};
    launches.push_back(L);
  }
  if (hdr.size() > kBatchListBytes) return ILS_ERR_WORKSPACE;
  for (size_t c = 0; c < launches.size(); ++c) {
    const FrameDesc* dd = reinterpret_cast<const FrameDesc*>(plan->ws + offs[4 * c]);
    launches[c].row.descs = dd;
    launches[c].fin.descs = dd;
    launches[c].col.descs = dd;
    launches[c].row.starts = reinterpret_cast<const int*>(plan->ws + offs[4 * c + 1]);
    launches[c].fin.starts = reinterpret_cast<const int*>(plan->ws + offs[4 * c + 2]);
    launches[c].col.starts = reinterpret_cast<const int*>(plan->ws + offs[4 * c + 3]);
    if (chs_offs[c] >= 0) launches[c].chs = reinterpret_cast<const int*>(plan->ws + chs_offs[c]);
  }
  hipError_t e = stage_upload(plan, plan->ws, hdr.data(), hdr.size());
  if (e != hipSuccess) return record(plan, e);

  // Chain `lane` on stream st: first its parts of large frames, each part's
  // whole 2N+1-pass sequence before the next part's; then its parts of
  // small frames in pass-major order (every part's pass k before any pass
  // k + 1).
  int maxN = 0;
  for (const Launch& L : launches) maxN = L.N > maxN ? L.N : maxN;
  // A part with a persistent launch runs its whole sequence in that one launch, in
  // the place of its first pass.
  auto persist_part = [&](const Launch& L, hipStream_t st) {
    return enqueue_persist(plan, L.fo, L.row.descs, L.chs, L.d0, L.row.n, L.C0, L.channels, L.N, L.pen, L.first,
                         L.ctl, st);
  };
  auto enqueue_chain = [&](int lane, hipStream_t st) -> hipError_t {
    hipError_t r = hipSuccess;
    for (const Launch& L : launches) {
      if (L.lane != lane || !L.big) continue;
      if (L.fo) {
        r = persist_part(L, st);
        if (r != hipSuccess) return r;
        continue;
      }
      r = timed(plan, 0, [&] { return L.pk.rv->launch(L.first, L.pen, L.row, st); });
      if (r != hipSuccess) return r;
      for (int n = 0; n < L.N; ++n) {
        r = timed(plan, 3, [&] { return L.pk.cv->launch(L.col, st); });
        if (r != hipSuccess) return r;
        if (n + 1 < L.N)
          r = timed(plan, 1, [&] { return L.pk.rv->launch(ilsk::ROW_MID, L.pen, L.row, st); });
        else
          r = timed(plan, 2, [&] { return L.pk.rv->launch(ilsk::ROW_FINAL, L.pen, L.fin, st); });
        if (r != hipSuccess) return r;
      }
    }
    for (const Launch& L : launches) {
      if (L.lane != lane || L.big) continue;
      if (L.fo)
        r = persist_part(L, st);
      else
        r = timed(plan, 0, [&] { return L.pk.rv->launch(L.first, L.pen, L.row, st); });
      if (r != hipSuccess) return r;
    }
    for (int n = 0; n < maxN; ++n) {
      for (const Launch& L : launches) {
        if (L.lane != lane || L.big || L.fo || n >= L.N) continue;
        r = timed(plan, 3, [&] { return L.pk.cv->launch(L.col, st); });
        if (r != hipSuccess) return r;
      }
      for (const Launch& L : launches) {
        if (L.lane != lane || L.big || L.fo || n >= L.N) continue;
        if (n + 1 < L.N)
          r = timed(plan, 1, [&] { return L.pk.rv->launch(ilsk::ROW_MID, L.pen, L.row, st); });
        else
          r = timed(plan, 2, [&] { return L.pk.rv->launch(ilsk::ROW_FINAL, L.pen, L.fin, st); });
        if (r != hipSuccess) return r;
      }
    }
    return r;
  };
  bool used[kChains] = {};
  for (const Launch& L : launches) used[L.lane] = true;
  // Without a graph (pass timing, ILS_PLAN_NO_GRAPH, or a batch of one part,
  // which has no second chain and only 2N + 1 launches): the chains one
  // after another on the caller's stream.
  if (plan->prof_on || !plan->cap_stream || launches.size() == 1) {
    for (int c = 0; c < kChains && e == hipSuccess; ++c) e = enqueue_chain(c, plan->stream);
    return record(plan, e);
  }

  // The whole 2N+1-pass sequence as one graph: the kernels read every frame
  // parameter from the work lists in the workspace header, so a replay for a
  // batch of the same structure needs no node updates.
  std::vector<long long> sig;
  sig.push_back((long long)hdr.size());
  for (const Launch& L : launches) {
    sig.push_back(L.lane);
    sig.push_back(L.big);
    sig.push_back((long long)(uintptr_t)L.pk.rv);
    sig.push_back((long long)(uintptr_t)L.pk.cv);
    sig.push_back(L.N);
    sig.push_back(L.pen);
    sig.push_back(L.first);
    sig.push_back(L.row.n);
    sig.push_back(L.row.total);
    sig.push_back(L.fin.total);
    sig.push_back(L.col.total);
    sig.push_back((long long)(uintptr_t)L.fo);
    sig.push_back((long long)(uintptr_t)L.ctl);
    sig.push_back((long long)(uintptr_t)L.chs);
  }
  for (size_t o : offs) sig.push_back((long long)o);
  size_t hit = 0;
  while (hit < plan->graphs.size() && plan->graphs[hit].sig != sig) ++hit;
  if (hit < plan->graphs.size()) {
    std::rotate(plan->graphs.begin(), plan->graphs.begin() + hit, plan->graphs.begin() + hit + 1);
  } else {
    if (plan->graphs.size() >= kGraphCache) {
      (void)hipGraphExecDestroy(plan->graphs.back().exec);
      plan->graphs.pop_back();
    }
    hipGraphExec_t exec = nullptr;
    hipGraph_t g = nullptr;
    e = hipStreamBeginCapture(plan->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return record(plan, e);
    // chains 1.. fork from the start of the capture and join before its
    // end, so the graph holds the chains as independent branches
    hipError_t el = hipEventRecord(plan->fork_ev, plan->cap_stream);
    for (int c = 1; c < kChains && el == hipSuccess; ++c)
      if (used[c]) el = hipStreamWaitEvent(plan->chain_stream[c], plan->fork_ev, 0);
    for (int c = 0; c < kChains && el == hipSuccess; ++c)
      if (used[c]) el = enqueue_chain(c, plan->chain_stream[c]);
    for (int c = 1; c < kChains && el == hipSuccess; ++c) {
      if (!used[c]) continue;
      el = hipEventRecord(plan->join_ev[c], plan->chain_stream[c]);
      if (el == hipSuccess) el = hipStreamWaitEvent(plan->cap_stream, plan->join_ev[c], 0);
    }
    e = hipStreamEndCapture(plan->cap_stream, &g);
    if (el != hipSuccess) e = el;
    if (e == hipSuccess) e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    if (e != hipSuccess) return record(plan, e);
    plan->graphs.insert(plan->graphs.begin(), ils_plan::BatchGraph{sig, exec});
  }
  return record(plan, hipGraphLaunch(plan->graphs.front().exec, plan->stream));
}

}  // extern "C"

// ------------------------------------------------- allocation-free variant
// Device memory of ils_smooth_noalloc: the tables of every compiled length
// (first kNoAllocTableBytes), then the two half spectra of one frame.  Each
// GPU the library runs on holds its own copy until the process ends.
constexpr size_t kNoAllocTableBytes = 4u << 20;
constexpr size_t kNoAllocBytes = 64u << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {
constexpr int kNoAllocDevices = 64;
struct NoAllocDevice {
  bool ready;
  char* base;  // device address of `scratch` on this device
  int cus;     // compute units (row banding)
  std::map<int, LenTables> tab;
};
NoAllocDevice g_noalloc[kNoAllocDevices];
std::mutex g_noalloc_mu;

// Set-up on the current device, once: the device address of `scratch`
// (host code must not use the array's name as an address) and the tables,
// copied into it synchronously.  Only this first call copies from the host.
int noalloc_device(NoAllocDevice** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return ILS_ERR_HIP;
  if (dev < 0 || dev >= kNoAllocDevices) return ILS_ERR_HIP;
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  NoAllocDevice& nd = g_noalloc[dev];
  if (!nd.ready) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return ILS_ERR_HIP;
    std::vector<char> host;
    std::map<int, LenTables> tab;
    build_tables(host, tab);
    if (host.size() > kNoAllocTableBytes) return ILS_ERR_HIP;
    if (hipMemcpy(ptr, host.data(), host.size(), hipMemcpyHostToDevice) != hipSuccess) return ILS_ERR_HIP;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 0;
    nd.cus = cus;
    nd.base = static_cast<char*>(ptr);
    nd.tab = std::move(tab);
    nd.ready = true;
  }
  *out = &nd;
  return ILS_OK;
}
}  // namespace

extern "C" {

size_t ils_noalloc_max_bytes(void) { return kNoAllocBytes - kNoAllocTableBytes; }

int ils_smooth_noalloc(const float* f, int H, int W, int C, float lambda, float p, float eps, int N, float* out,
                       void* hip_stream) {
  if (!f || !out) return ILS_ERR_INVALID_ARG;
  int rc = check_params(lambda, p, eps, N);
  if (rc != ILS_OK) return rc;
  rc = check_size(nullptr, H, W, C);
  if (rc != ILS_OK) return rc;
  if (frame_ws_bytes(H, W, C) > kNoAllocBytes - kNoAllocTableBytes) return ILS_ERR_WORKSPACE;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  if (N == 0 || lambda == 0.0f) {
    if (f == out) return ILS_OK;
    return hipMemcpyAsync(out, f, (size_t)C * H * W * sizeof(float), hipMemcpyDeviceToDevice, st) == hipSuccess
               ? ILS_OK
               : ILS_ERR_HIP;
  }
  NoAllocDevice* nd = nullptr;
  rc = noalloc_device(&nd);
  if (rc != ILS_OK) return rc;
  FrameDesc d;
  fill_desc_on(nd->base, nd->tab, d, H, W, C, lambda, p, eps);
  d.f = f;
  d.u0 = f;
  d.out = out;
  char* spec = nd->base + kNoAllocTableBytes;
  d.specA = reinterpret_cast<cf*>(spec);
  d.specB = reinterpret_cast<cf*>(spec + (size_t)C * H * d.ldS * sizeof(cf));
  // default tile shapes: no tuning (timing would create events)
  const Pick pk = default_pick(H, W);
  const hipError_t e =
      enqueue_frame(pk, d, N, ilsk::PEN_CHARBONNIER, nd->cus, st, [](int, auto&& launch) { return launch(); });
  return e == hipSuccess ? ILS_OK : ILS_ERR_HIP;
}

int ils_enqueue_pass(ils_plan* plan, int kind, const float* f, float* out, int H, int W, int C, float lambda,
                     float p, float eps) {
  if (!plan || !f || !out || kind < 0 || kind > 3) return ILS_ERR_INVALID_ARG;
  int rc = check_params(lambda, p, eps, 1);
  if (rc == ILS_OK) rc = check_size(plan, H, W, C);
  if (rc != ILS_OK) return rc;
  if (plan->ws_bytes < kBatchHeaderBytes + frame_ws_bytes(H, W, C)) return ILS_ERR_WORKSPACE;
  FrameDesc d;
  fill_desc(plan, d, H, W, C, lambda, p, eps);
  d.f = d.u0 = f;
  d.out = out;
  char* base = plan->ws + kBatchHeaderBytes;
  d.specA = reinterpret_cast<cf*>(base);
  d.specB = reinterpret_cast<cf*>(base + (size_t)C * H * d.ldS * sizeof(cf));
  const Pick pk = choose(plan, d);
  hipError_t e;
  if (kind == 3) {
    e = pk.cv->launch(one_frame(d, col_items(pk.cv, d)), plan->stream);
  } else {
    const int mode = kind == 0 ? ilsk::ROW_FIRST_SAME : kind == 1 ? ilsk::ROW_MID : ilsk::ROW_FINAL;
    const FrameDesc db = banded(plan->cus, pk.rv, d);
    e = pk.rv->launch(mode, ilsk::PEN_CHARBONNIER, one_frame(db, row_items(pk.rv, mode, db)), plan->stream);
  }
  return record(plan, e);
}

// ------------------------------------------------------------ debug passes
int ils_debug_rhs_spectrum(ils_plan* plan, const float* f, const float* u0, int H, int W, int C,
                           float lambda, float p, float eps, float* spec) {
  if (!plan || !f || !u0 || !spec) return ILS_ERR_INVALID_ARG;
  int rc = check_params(lambda, p, eps, 1);
  if (rc == ILS_OK) rc = check_size(plan, H, W, C);
  if (rc != ILS_OK) return rc;
  if (plan->ws_bytes < kBatchHeaderBytes + frame_ws_bytes(H, W, C)) return ILS_ERR_WORKSPACE;
  FrameDesc d;
  fill_desc(plan, d, H, W, C, lambda, p, eps);
  d.f = f;
  d.u0 = u0;
  d.out = nullptr;
  char* base = plan->ws + kBatchHeaderBytes;
  d.specA = reinterpret_cast<cf*>(base);
  d.specB = reinterpret_cast<cf*>(base + (size_t)C * H * d.ldS * sizeof(cf));
  // the runtime-length first pass writes the second half spectrum
  const RowVariant* v = default_pick(H, W).rv;
  const cf* res = frame_generic(H, W) ? d.specB : d.specA;
  hipError_t e = v->launch(ilsk::ROW_FIRST, ilsk::PEN_CHARBONNIER, one_frame(d, row_items(v, ilsk::ROW_FIRST, d)), plan->stream);
  if (e == hipSuccess)
    e = hipMemcpy2DAsync(spec, (size_t)(W / 2 + 1) * sizeof(cf), res, (size_t)d.ldS * sizeof(cf),
                         (size_t)(W / 2 + 1) * sizeof(cf), (size_t)C * H, hipMemcpyDeviceToDevice,
                         plan->stream);
  return record(plan, e);
}

int ils_debug_column_solve(ils_plan* plan, const float* spec_in, int H, int W, int C, float lambda,
                           float p, float eps, float* spec_out) {
  if (!plan || !spec_in || !spec_out) return ILS_ERR_INVALID_ARG;
  int rc = check_params(lambda, p, eps, 1);
  if (rc == ILS_OK) rc = check_size(plan, H, W, C);
  if (rc != ILS_OK) return rc;
  if (plan->ws_bytes < kBatchHeaderBytes + frame_ws_bytes(H, W, C)) return ILS_ERR_WORKSPACE;
  FrameDesc d;
  fill_desc(plan, d, H, W, C, lambda, p, eps);
  d.f = d.u0 = nullptr;
  d.out = nullptr;
  char* base = plan->ws + kBatchHeaderBytes;
  d.specA = reinterpret_cast<cf*>(base);
  d.specB = reinterpret_cast<cf*>(base + (size_t)C * H * d.ldS * sizeof(cf));
  const size_t rowb = (size_t)(W / 2 + 1) * sizeof(cf);
  // the runtime-length column pass works in place on the second half spectrum
  cf* in = frame_generic(H, W) ? d.specB : d.specA;
  hipError_t e = hipMemcpy2DAsync(in, (size_t)d.ldS * sizeof(cf), spec_in, rowb, rowb,
                                  (size_t)C * H, hipMemcpyDeviceToDevice, plan->stream);
  const ColVariant* cv = default_pick(H, W).cv;
  if (e == hipSuccess) e = cv->launch(one_frame(d, col_items(cv, d)), plan->stream);
  if (e == hipSuccess)
    e = hipMemcpy2DAsync(spec_out, rowb, d.specB, (size_t)d.ldS * sizeof(cf), rowb, (size_t)C * H,
                         hipMemcpyDeviceToDevice, plan->stream);
  return record(plan, e);
}

int ils_debug_row_inverse(ils_plan* plan, const float* spec, int H, int W, int C, float* out) {
  if (!plan || !spec || !out) return ILS_ERR_INVALID_ARG;
  int rc = check_size(plan, H, W, C);
  if (rc != ILS_OK) return rc;
  if (plan->ws_bytes < kBatchHeaderBytes + frame_ws_bytes(H, W, C)) return ILS_ERR_WORKSPACE;
  FrameDesc d;
  fill_desc(plan, d, H, W, C, 1.0f, 1.0f, 1e-4f);
  d.f = d.u0 = nullptr;
  d.out = out;
  char* base = plan->ws + kBatchHeaderBytes;
  d.specA = reinterpret_cast<cf*>(base + (size_t)C * H * d.ldS * sizeof(cf));
  d.specB = reinterpret_cast<cf*>(base);
  const size_t rowb = (size_t)(W / 2 + 1) * sizeof(cf);
  hipError_t e = hipMemcpy2DAsync(d.specB, (size_t)d.ldS * sizeof(cf), spec, rowb, rowb, (size_t)C * H,
                                  hipMemcpyDeviceToDevice, plan->stream);
  const RowVariant* v = default_pick(H, W).rv;
  if (e == hipSuccess) e = v->launch(ilsk::ROW_FINAL, ilsk::PEN_CHARBONNIER, one_frame(d, row_items(v, ilsk::ROW_FINAL, d)), plan->stream);
  return record(plan, e);
}

}  // extern "C"

// Scratch area for small auxiliary kernels (the batch header region of the
// workspace; stream order separates its users).
int ilsk_plan_scratch(ils_plan* plan, void** scratch, size_t* bytes, void** stream) {
  if (!plan) return ILS_ERR_INVALID_ARG;
  *scratch = plan->ws;
  *bytes = kBatchHeaderBytes;
  *stream = plan->stream;
  return ILS_OK;
}

int ilsk_plan_upload(ils_plan* plan, void* dst, const void* src, size_t bytes) {
  return record(plan, stage_upload(plan, dst, src, bytes));
}

void* ilsk_plan_stream(ils_plan* plan) { return plan ? static_cast<void*>(plan->stream) : nullptr; }
