// The two fused passes of one ILS iteration (Algorithm 1), as device bodies.
//
// Row pass (band of G output rows of one channel):
//   MID   : spectrum rows y0-1 .. y0+G  --C2R-->  u^n rows (LDS)
//           stencil: forward differences, mu (Eq. (7)), adjoint differences
//           r = f + kappa * D^T mu                     (Eq. (9) numerator,
//                                                       one-FFT form, Sec. 3.2)
//           r rows y0 .. y0+G-1  --R2C-->  spectrum rows
//   FIRST : as MID with u^0 rows read from memory instead of the C2R
//   FINAL : spectrum rows --C2R--> u^N rows written to the output
// Column pass (tile of S spectrum columns of one channel):
//   forward column DFT, divide by 1 + kappa (Sx + Sy) (Eq. (9) denominator)
//   and the inverse normalisation, inverse column DFT.
//
// A length-M complex DFT is split M = P * Q (four-step): the element index
// n = Q n1 + t is held by lane t (register n1) in "spatial" layout; stage A
// is a P-point register DFT per lane, a twiddle exp(-+2 pi i t k1 / M), one
// LDS exchange, and stage B a Q-point register DFT per lane k1, giving
// X[k1 + P k2] in register k2.  The inverse runs the same steps backwards,
// so no digit reversal is ever materialised.
#pragma once

#include "fft_reg.hpp"
#include "ils_desc.hpp"

namespace ilsk {

__device__ __forceinline__ int imax(int a, int b) { return a > b ? a : b; }
__device__ __forceinline__ int imin(int a, int b) { return a < b ? a : b; }

// Normalised half-quadratic variable  mu / c = g (1 - (c0/c) (1 + g^2/eps)^(p/2 - 1))
// (Eq. (7) divided by c, c0 = p eps^(p/2-1)); base-2 log/exp on the hardware
// transcendental unit.  l2r = log2(c0 / c) is 0 for c = c0.
__device__ __forceinline__ float mu_ns(float g, float a_exp, float inv_eps, float l2r) {
  float t = fmaf(g * g, inv_eps, 1.0f);
  float pw = __builtin_amdgcn_exp2f(fmaf(a_exp, __builtin_amdgcn_logf(t), l2r));
  return fmaf(-g, pw, g);
}

// Welsch penalty (Sec. 5, Eqs. (18)-(20)): with c = c0 = 2 the normalised
// variable is mu / c = g (1 - exp(-g^2 / (2 gamma^2))); w = -log2(e) / (2 gamma^2).
__device__ __forceinline__ float mu_ns_welsch(float g, float w, float l2r) {
  return fmaf(-g, __builtin_amdgcn_exp2f(fmaf(w, g * g, l2r)), g);
}

enum Penalty : int { PEN_CHARBONNIER = 0, PEN_WELSCH = 1 };

// mu / c for the penalty of the kernel instance: (a, b) = (p/2 - 1, 1/eps)
// for the generalised Charbonnier penalty, (w, unused) for Welsch; l2r =
// log2(c0 / c).
template <int PEN>
__device__ __forceinline__ float mu_pen(float g, float a, float b, float l2r) {
  if constexpr (PEN == PEN_WELSCH)
    return mu_ns_welsch(g, a, l2r);
  else
    return mu_ns(g, a, b, l2r);
}

// Cross-lane moves inside a wavefront (no LDS allocation): the value of the
// previous lane (a DPP wave shift), and the value of the last lane of a
// T-lane slot broadcast to the whole slot (ds_swizzle bit mode, within
// 32-lane groups; T a power of two <= 32).
__device__ __forceinline__ float from_prev_lane(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138 /* wave_shr:1 */, 0xf, 0xf, false));
}
__device__ __forceinline__ float from_next_lane(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130 /* wave_shl:1 */, 0xf, 0xf, false));
}
// the value of the first lane of a T-lane slot (ds_swizzle bit mode)
template <int T>
__device__ __forceinline__ float from_slot_first_lane(float v) {
  static_assert(T <= 32 && (T & (T - 1)) == 0, "slot must be a power of two within 32 lanes");
  constexpr int pattern = 31 & ~(T - 1);  // and-mask, or-mask 0, xor-mask 0
  return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), pattern));
}
template <int T>
__device__ __forceinline__ float from_slot_last_lane(float v) {
  static_assert(T <= 32 && (T & (T - 1)) == 0, "slot must be a power of two within 32 lanes");
  constexpr int pattern = (31 & ~(T - 1)) | ((T - 1) << 5);  // and-mask, or-mask, xor-mask 0
  return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), pattern));
}

// Synchronisation inside one row slot.  When a slot lies within one
// wavefront (T divides 64) its LDS exchange needs no workgroup barrier: the
// LDS operations of a wavefront are performed in program order, so it is
// enough to keep the compiler from moving memory operations across this
// point.  Otherwise fall back to a workgroup barrier.
template <int T>
__device__ __forceinline__ void slot_sync() {
  if constexpr (64 % T == 0) {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
  } else {
    __syncthreads();
  }
}

template <int P, int Q>
struct RowGeom {
  static constexpr int M = P * Q;
  static constexpr int T = P > Q ? P : Q;    // lanes per row slot
  static constexpr int QP = Q | 1;           // padded exchange row (odd => conflict-free)
  static constexpr int SLOT_F = 2 * P * QP;  // floats of LDS per row slot (>= W)
  static constexpr int TAB_F = 2 * P * QP;   // twiddles exp(-2 pi i t k1 / M) at [k1][t]
  static constexpr int NPOST = (M + 1 + T - 1) / T;  // post-process elements per lane
};

// LDS that co-resident workgroups of one kernel may take on a CU in all.  A
// single workgroup may use the whole 160 KB, but two are placed on one CU
// only when each takes at most about 77 KB (measured on MI355X: two blocks
// of 77 280 B run side by side, two of 79 200 B do not).
constexpr int kLdsCoresident = 154560;
constexpr int resident_blocks(int lds_bytes) {
  return lds_bytes * 2 > kLdsCoresident ? 1 : kLdsCoresident / lds_bytes;
}

// Waves per SIMD that the workgroups resident on a CU (as many as fit its
// LDS, at most 8 per SIMD) need; each may then use 512 / waves VGPRs.
constexpr int resident_waves_per_simd(int threads, int lds_bytes) {
  const int blocks = resident_blocks(lds_bytes);
  const int waves = blocks * ((threads + 63) / 64);
  return (waves + 3) / 4 > 8 ? 8 : (waves + 3) / 4;
}
template <int P, int Q, int G>
constexpr int row_waves() {
  return resident_waves_per_simd((G + 2) * RowGeom<P, Q>::T, 4 * ((G + 2) * RowGeom<P, Q>::SLOT_F + RowGeom<P, Q>::TAB_F));
}

// Rows per row-pass workgroup: about half the LDS of a CU when that leaves
// bands of at least four rows, else all of it.
template <int P, int Q>
constexpr int row_band() {
  constexpr int slot = 4 * RowGeom<P, Q>::SLOT_F;
  constexpr int tab = 4 * RowGeom<P, Q>::TAB_F;
  int g = (81920 - tab) / slot - 2;
  if (g < 4) g = (163840 - tab) / slot - 2;
  if (g > 14) g = 14;
  if (g < 1) g = 1;
  return g;
}

// Alternatives offered to the tuner: one workgroup per CU with the largest
// band that fits (fewest halo rows per output row), bands of about 3/4 and
// 5/8 of it, which split a frame into fewer blocks than CUs more evenly, and
// bands of 5 and 4 rows for frames with few rows in all.
template <int P, int Q>
constexpr int row_band_max() {
  constexpr int slot = 4 * RowGeom<P, Q>::SLOT_F;
  constexpr int tab = 4 * RowGeom<P, Q>::TAB_F;
  int g = (163840 - tab) / slot - 2;
  if (g > 30) g = 30;
  while ((g + 2) * RowGeom<P, Q>::T > 1024) --g;
  if (g < 1) g = 1;
  return g;
}
template <int P, int Q, int i>
constexpr int row_band_alt() {
  constexpr int gm = row_band_max<P, Q>();
  // i = 3, 4: short bands (5 and 4 rows) that spread a one-channel frame
  // over all CUs
  return i == 0 ? gm : i == 1 ? (3 * gm + 2) / 4 : i == 2 ? (5 * gm + 4) / 8 : i == 3 ? 5 : 4;
}

// Column tile of S spectrum columns.  The exchange row of one k1 is padded
// so that successive k1 groups land on different LDS banks.
constexpr int col_ks(int Q, int S) { return (S >= 16) ? Q * S : Q * S + ((S - (Q * S) % 16) + 16) % 16; }
constexpr int col_ex_f(int P, int Q, int S) { return 2 * P * col_ks(Q, S); }
constexpr bool col_fits(int P, int Q, int S, int tab_f) {
  return 4 * (col_ex_f(P, Q, S) + tab_f) <= 163840 && S * (P > Q ? P : Q) <= 1024;
}

// Tables of a column length: the twiddles as a P x (Q|1) matrix [k1][j]
// and Sy[l] = 4 sin^2(pi l / H).  A tile copies them into its LDS beside the
// exchange when that costs no resident block on a CU; otherwise (the tiles
// of the longest columns) it reads them from global memory, where every
// block of the length finds them in the cache.  Either way every tile width
// of a length computes the same bits.
template <int P, int Q, int S>
struct ColGeom {
  static constexpr int H = P * Q;
  static constexpr int T = P > Q ? P : Q;
  static constexpr int QT = Q | 1;  // row stride of the twiddle matrix
  static constexpr int KS = col_ks(Q, S);
  static constexpr int EX_F = col_ex_f(P, Q, S);
  static constexpr int TAB_F = 2 * P * QT + H;
  static constexpr bool fits = col_fits(P, Q, S, 0);
  static constexpr bool TAB_LDS =
      col_fits(P, Q, S, TAB_F) && resident_blocks(4 * (EX_F + TAB_F)) == resident_blocks(4 * EX_F);
  static constexpr int LDS_F = EX_F + (TAB_LDS ? TAB_F : 0);
};

// Default column tile: the widest whose exchange and table fit the 160 KB of
// LDS (16 columns are whole 128-byte lines of the row-major spectrum;
// narrower tiles make neighbouring blocks fetch the same lines).  The
// narrower tiles offered to the tuner trade line efficiency for a grid that
// spreads more evenly over the compute units.
template <int P, int Q>
constexpr int col_tile() {
  return ColGeom<P, Q, 16>::fits ? 16 : ColGeom<P, Q, 8>::fits ? 8 : 4;
}
template <int P, int Q, int i>
constexpr int col_tile_alt() {
  constexpr int w = col_tile<P, Q>();
  constexpr int cand[3] = {w == 16 ? 12 : 4, 8, 4};
  return ColGeom<P, Q, cand[i]>::fits && cand[i] < w ? cand[i] : w;
}

// exp(+- i pi m / n) as a compile-time complex constant.
template <long long m, long long n>
__device__ __forceinline__ cf turn_half() {
  constexpr dcs w = cossin_turn(m, 2 * n);
  return cf{float(w.c), float(w.s)};
}

// ---- C2R stage A' of one row (lane k1 < P): pre-process X[k], X[M-k] into
// Z[k] = (X[k] + conj X[M-k]) + i (X[k] - conj X[M-k]) exp(i pi k / M) and
// take the Q-point inverse DFT over k2 (k = k1 + P k2); c2r_exchange then
// applies the twiddle exp(2 pi i t k1 / M) and writes the exchange row
// [k1][t].
template <int P, int Q>
__device__ __forceinline__ void c2r_stage_a(const ILS_G cf* X, int k1, cf w1, cf (&v)[Q]) {
  constexpr int M = P * Q;
  static_for<Q>([&](auto k2c) {
    constexpr int k2 = decltype(k2c)::value;
    const int k = k1 + P * k2;
    cf a = X[k];
    cf b = X[M - k];
    if (k2 == 0 && k1 == 0) {  // DC and Nyquist bins: real parts only
      a.y = 0.0f;
      b.y = 0.0f;
    }
    const cf bc = {b.x, -b.y};
    const cf e = cadd(a, bc);
    // exp(i pi k / M) = exp(i pi k1 / M) exp(i pi k2 / Q)
    const cf wk = (k2 == 0) ? w1 : cmul(w1, turn_half<k2, Q>());
    const cf o = cmul(csub(a, bc), wk);
    v[k2] = {e.x - o.y, e.y + o.x};  // e + i o
  });
  dft<Q, +1>(v);
}

// twiddle exp(2 pi i t k1 / M) from the LDS table, then the exchange row [k1][t]
// (All table reads are issued before the first exchange write: the table and
// the exchange share one LDS array, so interleaving them would serialise.)
template <int P, int Q>
__device__ __forceinline__ void c2r_exchange(const cf (&v)[Q], int k1, const cf* tws, cf* slc) {
  constexpr int QP = Q | 1;
  cf w[Q];
  const cf* wrow = tws + k1 * QP;
  static_for<Q>([&](auto tc) {
    constexpr int t = decltype(tc)::value;
    if constexpr (t > 0) w[t] = wrow[t];
  });
  static_for<Q>([&](auto tc) {
    constexpr int t = decltype(tc)::value;
    slc[k1 * QP + t] = (t == 0) ? v[t] : cmulc(v[t], w[t]);
  });
}

// ---- C2R stage B' (lane t < Q): P-point inverse DFT over k1 -> z[Q n1 + t].
template <int P, int Q>
__device__ __forceinline__ void c2r_stage_b(const cf* slc, int t, cf (&z)[P]) {
  constexpr int QP = Q | 1;
  static_for<P>([&](auto k1c) {
    constexpr int k1 = decltype(k1c)::value;
    z[k1] = slc[k1 * QP + t];
  });
  dft<P, +1>(z);
}

// ---- R2C post-process of one row held in LDS in natural order Z[0..M-1]:
// X'[k] = E - i W_2M^k D with E = Z[k] + conj Z[M-k], D = Z[k] - conj Z[M-k]
// (X' = 2 X), k = lane + T i <= M;  W_2M^k = W_2M^lane * W_2M^(T i).
template <int P, int Q>
__device__ __forceinline__ void r2c_post(const cf* slc, int lane, cf wl, ILS_G cf* Xo) {
  using Geo = RowGeom<P, Q>;
  constexpr int M = Geo::M, T = Geo::T;
  // every element but the last is in range (T (NPOST - 1) <= M), so only the
  // last one is guarded and the rest stays one basic block
  auto one = [&](auto ic) {
    constexpr int i = decltype(ic)::value;
    const int k = lane + T * i;
    cf A = slc[k == M ? 0 : k];
    cf B = slc[k == 0 ? 0 : M - k];
    B.y = -B.y;
    const cf E = cadd(A, B), D = csub(A, B);
    const cf w = (i == 0) ? wl : cmul(wl, turn_half<-(long long)T * i, M>());
    const cf wD = cmul(D, w);
    Xo[k] = {E.x + wD.y, E.y - wD.x};  // E - i wD
  };
  static_for<Geo::NPOST - 1>(one);
  if (lane + T * (Geo::NPOST - 1) <= M) one(std::integral_constant<int, Geo::NPOST - 1>{});
}

// --------------------------------------------------------------------------
// Row pass, modes FIRST and MID.  Block = (G + 2) slots x T lanes.
// Slot s holds row y0 - 1 + s (periodic), s = 0 .. Gv + 1.
// LDS: (G + 2) slots of SLOT_F floats, then the twiddle table.
// --------------------------------------------------------------------------
template <int P, int Q, int G, int MODE, int PEN>
__device__ __forceinline__ void row_body(const FrameDesc& d, int band, int ch, float* smem) {
  using Geo = RowGeom<P, Q>;
  constexpr int M = Geo::M, T = Geo::T, QP = Geo::QP, SLOT_F = Geo::SLOT_F;
  const int H = d.H;
  const int W = 2 * M;
  const int ldS = d.ldS;
  const int nb = row_bands(d, G);
  const int y0 = band * H / nb;
  const int Gv = (band + 1) * H / nb - y0;
  const int tid = threadIdx.x;
  const int slot = tid / T;
  const int lane = tid - slot * T;
  float* sl = smem + slot * SLOT_F;
  cf* slc = reinterpret_cast<cf*>(sl);
  cf* tws = reinterpret_cast<cf*>(smem + (G + 2) * SLOT_F);
  const bool in_slot = slot <= Gv + 1;
  int yrow = y0 - 1 + slot;
  yrow = yrow < 0 ? yrow + H : (yrow >= H ? yrow - H : yrow);
  if (!in_slot) yrow = 0;
  const bool out_slot = slot >= 1 && slot <= Gv;
  const int yout = out_slot ? y0 - 1 + slot : 0;
  const ILS_G float2* frow = reinterpret_cast<const ILS_G float2*>(gm(d.f) + (size_t)ch * H * W + (size_t)yout * W);

  // per-lane factors of the real-FFT twiddles (one load each, issued first)
  const cf w2lane = gm(d.tw2_row)[lane];  // exp(-i pi lane / M)
  // twiddle table -> LDS
  for (int i = tid; i < P * Geo::QP; i += blockDim.x) tws[i] = gm(d.twm_row)[i];

  float2 fv[P];
  // u^0 = f (Algorithm 1): the data term is the slot's own u row
  constexpr bool f_is_u0 = (MODE == ROW_FIRST_SAME);
  // When a slot is Q lanes of one wavefront (Q a power of two), mu_x is
  // passed between lanes (below).  If moreover the shape leaves 256 VGPRs
  // per lane (two waves per SIMD), each lane keeps its own pairs of u in
  // registers for the stencil and takes the right neighbour from the next
  // lane; only the row below comes from LDS.  Both read the same values.
  constexpr bool kLaneReuse = (T == Q) && (T <= 32) && ((T & (T - 1)) == 0);
  constexpr bool kRegRow = kLaneReuse && row_waves<P, Q, G>() <= 2;
  float2 ur[P];
  if constexpr (MODE == ROW_FIRST || MODE == ROW_FIRST_SAME) {
    if (in_slot && lane < Q) {  // u^0 row of this slot, all loads in flight together
      const ILS_G float2* urow = reinterpret_cast<const ILS_G float2*>(gm(d.u0) + (size_t)ch * H * W + (size_t)yrow * W);
      float2 uv[P];
      static_for<P>([&](auto n1c) {
        constexpr int n1 = decltype(n1c)::value;
        uv[n1] = urow[Q * n1 + lane];
      });
      if (out_slot && !f_is_u0) {
        static_for<P>([&](auto n1c) {
          constexpr int n1 = decltype(n1c)::value;
          fv[n1] = frow[Q * n1 + lane];
        });
      }
      float2* u2 = reinterpret_cast<float2*>(sl);
      static_for<P>([&](auto n1c) {
        constexpr int n1 = decltype(n1c)::value;
        u2[Q * n1 + lane] = uv[n1];
        if constexpr (kRegRow) ur[n1] = uv[n1];
      });
    }
    __syncthreads();
  } else {
    // ---- C2R of this slot's row (its loads overlap the table load)
    cf v[Q];
    if (in_slot && lane < P) {
      const ILS_G cf* X = gm(d.specB) + (size_t)ch * H * ldS + (size_t)yrow * ldS;
      c2r_stage_a<P, Q>(X, lane, cf{w2lane.x, -w2lane.y}, v);
    }
    __syncthreads();  // twiddle table ready
    if (in_slot && lane < P) c2r_exchange<P, Q>(v, lane, tws, slc);
    if (out_slot && lane < Q) {  // data term, in flight during stage B'
      static_for<P>([&](auto n1c) {
        constexpr int n1 = decltype(n1c)::value;
        fv[n1] = frow[Q * n1 + lane];
      });
    }
    slot_sync<T>();
    cf z[P];
    if (in_slot && lane < Q) c2r_stage_b<P, Q>(slc, lane, z);
    slot_sync<T>();
    if (in_slot && lane < Q) {
      float2* u2 = reinterpret_cast<float2*>(sl);
      static_for<P>([&](auto n1c) {
        constexpr int n1 = decltype(n1c)::value;
        u2[Q * n1 + lane] = make_float2(z[n1].x, z[n1].y);
        if constexpr (kRegRow) ur[n1] = make_float2(z[n1].x, z[n1].y);
      });
    }
    __syncthreads();
  }

  // ---- stencil.  mu_y of row s (from rows s, s+1) is evaluated once by
  // slot s and handed to slot s+1 through LDS; mu_x at x-1 is re-evaluated
  // locally.  Slot 0 (the row above the band) only supplies mu_y.
  const int t = lane;
  cf r[P];
  float2 myd[P];
  const bool st_slot = slot <= Gv && lane < Q;  // slots 0..Gv evaluate mu_y
  if (st_slot) {
    const float2* uc = reinterpret_cast<const float2*>(sl);
    const float2* ud = reinterpret_cast<const float2*>(sl + SLOT_F);
    const float a_exp = d.a_exp, inv_eps = d.inv_eps, kappa = d.kappa, l2r = d.log2_r;
    if (slot >= 1) {
      // mu_x left of pair j equals mu_x right of pair j - 1.  When a slot is
      // Q lanes of one wavefront, pair j - 1 sits in the previous lane (same
      // n1) or, for lane 0, in lane Q - 1 at n1 - 1: take it from there.
      // Likewise pair j + 1 (the right neighbour's first pixel) sits in the
      // next lane, or for lane Q - 1 in lane 0 at n1 + 1 (at n1 = P - 1 that
      // is pair 0, the periodic wrap).
      float mx1_prev = 0.0f;
      static_for<P>([&](auto n1c) {
        constexpr int n1 = decltype(n1c)::value;
        const int j = Q * n1 + t;
        const int jp = (j == M - 1) ? 0 : j + 1;
        float2 c, rr;
        if constexpr (kRegRow) {
          c = ur[n1];
          constexpr int n1n = (n1 + 1) % P;
          const float nx = from_next_lane(c.x);
          const float wx = from_slot_first_lane<T>(ur[n1n].x);
          rr.x = (t == Q - 1) ? wx : nx;
          rr.y = 0.0f;
        } else {
          c = uc[j];
          rr = uc[jp];
        }
        const float2 dn = ud[j];
        if (f_is_u0) fv[n1] = c;
        myd[n1] = make_float2(mu_pen<PEN>(dn.x - c.x, a_exp, inv_eps, l2r), mu_pen<PEN>(dn.y - c.y, a_exp, inv_eps, l2r));
        const float mx0 = mu_pen<PEN>(c.y - c.x, a_exp, inv_eps, l2r);
        const float mx1 = mu_pen<PEN>(rr.x - c.y, a_exp, inv_eps, l2r);
        float mxl;
        if constexpr (kLaneReuse && n1 > 0) {
          const float sh = from_prev_lane(mx1);
          const float wr = from_slot_last_lane<T>(mx1_prev);
          mxl = (t == 0) ? wr : sh;
        } else {
          const int jm = (j == 0) ? M - 1 : j - 1;
          mxl = mu_pen<PEN>(c.x - uc[jm].y, a_exp, inv_eps, l2r);
        }
        mx1_prev = mx1;
        r[n1] = {fmaf(kappa, (mxl - mx0) - myd[n1].x, fv[n1].x), fmaf(kappa, (mx0 - mx1) - myd[n1].y, fv[n1].y)};
        // batches of five positions: their LDS reads issue together, while
        // the registers of later positions are not claimed early
        if constexpr ((n1 + 1) % 5 == 0) __builtin_amdgcn_sched_barrier(0);
      });
    } else {
      static_for<P>([&](auto n1c) {
        constexpr int n1 = decltype(n1c)::value;
        const int j = Q * n1 + t;
        float2 c;
        if constexpr (kRegRow)
          c = ur[n1];
        else
          c = uc[j];
        const float2 dn = ud[j];
        myd[n1] = make_float2(mu_pen<PEN>(dn.x - c.x, a_exp, inv_eps, l2r), mu_pen<PEN>(dn.y - c.y, a_exp, inv_eps, l2r));
      });
    }
  }
  __syncthreads();  // every read of u done
  if (st_slot && slot < Gv) {
    float2* md = reinterpret_cast<float2*>(sl);
    static_for<P>([&](auto n1c) {
      constexpr int n1 = decltype(n1c)::value;
      md[Q * n1 + t] = myd[n1];
    });
  }
  __syncthreads();
  // ---- add mu_y of the row above, then stage A (P-point forward)
  if (out_slot && lane < Q) {
    const float2* mu = reinterpret_cast<const float2*>(sl - SLOT_F);
    const float kappa = d.kappa;
    static_for<P>([&](auto n1c) {
      constexpr int n1 = decltype(n1c)::value;
      const float2 m = mu[Q * n1 + t];
      r[n1] = {fmaf(kappa, m.x, r[n1].x), fmaf(kappa, m.y, r[n1].y)};
    });
    dft<P, -1>(r);
    static_for<P>([&](auto k1c) {
      constexpr int k1 = decltype(k1c)::value;
      if (k1 != 0) r[k1] = cmul(r[k1], tws[k1 * QP + t]);
    });
  }
  __syncthreads();
  if (out_slot && lane < Q) {
    static_for<P>([&](auto k1c) {
      constexpr int k1 = decltype(k1c)::value;
      slc[k1 * QP + lane] = r[k1];
    });
  }
  slot_sync<T>();
  cf zz[Q];
  if (out_slot && lane < P) {
    const int k1 = lane;
    static_for<Q>([&](auto tc) {
      constexpr int t = decltype(tc)::value;
      zz[t] = slc[k1 * QP + t];
    });
    dft<Q, -1>(zz);
  }
  slot_sync<T>();
  if (out_slot && lane < P) {
    const int k1 = lane;
    static_for<Q>([&](auto k2c) {
      constexpr int k2 = decltype(k2c)::value;
      slc[k1 + P * k2] = zz[k2];
    });
  }
  slot_sync<T>();
  if (out_slot) r2c_post<P, Q>(slc, lane, w2lane, gm(d.specA) + (size_t)ch * H * ldS + (size_t)yout * ldS);
}

// --------------------------------------------------------------------------
// Row pass, mode FINAL: C2R of G rows, written to the output image.
// Block = G slots x T lanes; slot s holds row y0 + s.
// --------------------------------------------------------------------------
template <int P, int Q, int G>
__device__ __forceinline__ void row_final_body(const FrameDesc& d, int band, int ch, float* smem) {
  using Geo = RowGeom<P, Q>;
  constexpr int M = Geo::M, T = Geo::T, SLOT_F = Geo::SLOT_F;
  const int H = d.H;
  const int W = 2 * M;
  const int ldS = d.ldS;
  const int nb = row_bands(d, G);
  const int y0 = band * H / nb;
  const int Gv = (band + 1) * H / nb - y0;
  const int tid = threadIdx.x;
  const int slot = tid / T;
  const int lane = tid - slot * T;
  cf* slc = reinterpret_cast<cf*>(smem + slot * SLOT_F);
  cf* tws = reinterpret_cast<cf*>(smem + G * SLOT_F);
  const bool in_slot = slot < Gv;
  const int yrow = in_slot ? y0 + slot : 0;
  const cf w2lane = gm(d.tw2_row)[lane];
  for (int i = tid; i < P * Geo::QP; i += blockDim.x) tws[i] = gm(d.twm_row)[i];
  cf v[Q];
  if (in_slot && lane < P) {
    const ILS_G cf* X = gm(d.specB) + (size_t)ch * H * ldS + (size_t)yrow * ldS;
    c2r_stage_a<P, Q>(X, lane, cf{w2lane.x, -w2lane.y}, v);
  }
  __syncthreads();  // twiddle table ready
  if (in_slot && lane < P) c2r_exchange<P, Q>(v, lane, tws, slc);
  slot_sync<T>();
  if (in_slot && lane < Q) {
    cf z[P];
    c2r_stage_b<P, Q>(slc, lane, z);
    ILS_G float2* orow = reinterpret_cast<ILS_G float2*>(gm(d.out) + (size_t)ch * H * W + (size_t)yrow * W);
    const float k = d.boost;
    if (k != 0.0f) {  // detail enhancement: u + k (f - u); each element is read before it is written
      const ILS_G float2* frow = reinterpret_cast<const ILS_G float2*>(gm(d.f) + (size_t)ch * H * W + (size_t)yrow * W);
      static_for<P>([&](auto n1c) {
        constexpr int n1 = decltype(n1c)::value;
        const float2 fv = frow[Q * n1 + lane];
        orow[Q * n1 + lane] = make_float2(fmaf(k, fv.x - z[n1].x, z[n1].x), fmaf(k, fv.y - z[n1].y, z[n1].y));
      });
    } else {
      static_for<P>([&](auto n1c) {
        constexpr int n1 = decltype(n1c)::value;
        orow[Q * n1 + lane] = make_float2(z[n1].x, z[n1].y);
      });
    }
  }
}

// --------------------------------------------------------------------------
// Column pass.  Block = S columns x T lanes, lane id = s + S * j.
// LDS: exchange (P x KS complex), then the tables (twiddle matrix [k1][j],
// row stride Q|1, and Sy[l]) when they are kept in LDS.
// --------------------------------------------------------------------------
template <int P, int Q, int S_>
__device__ __forceinline__ void col_body(const FrameDesc& d, int tile, int ch, float* smem) {
  using Geo = ColGeom<P, Q, S_>;
  constexpr int H = Geo::H, S = S_, KS = Geo::KS, QT = Geo::QT;
  const int ldS = d.ldS;
  const int Wh = d.W / 2 + 1;
  const int tid = threadIdx.x;
  const int s = tid % S;
  const int j = tid / S;
  const int c = tile * S + s;
  const bool col_ok = c < Wh;
  const int cc = col_ok ? c : 0;
  const ILS_G cf* in = gm(d.specA) + (size_t)ch * H * ldS + cc;
  ILS_G cf* out = gm(d.specB) + (size_t)ch * H * ldS + cc;
  cf* ex = reinterpret_cast<cf*>(smem);
  cf* tws = reinterpret_cast<cf*>(smem + Geo::EX_F);  // LDS copy of the twiddle matrix
  float* syl = smem + Geo::EX_F + 2 * P * QT;          // LDS copy of Sy
  const ILS_G cf* gtw = gm(d.twm_col);
  const ILS_G float* gsy = gm(d.sy);
  auto tw = [&](int i) -> cf {
    if constexpr (Geo::TAB_LDS)
      return tws[i];
    else
      return cf(gtw[i]);
  };
  auto sy_at = [&](int l) -> float {
    if constexpr (Geo::TAB_LDS)
      return syl[l];
    else
      return gsy[l];
  };

  cf x[P];
  if (j < Q) {  // stage A loads first: lane n2 = j, rows Q n1 + n2
    static_for<P>([&](auto n1c) {
      constexpr int n1 = decltype(n1c)::value;
      x[n1] = col_ok ? cf(in[(size_t)(Q * n1 + j) * ldS]) : cf{0.0f, 0.0f};
    });
  }
  const float sxk = gm(d.sx)[cc];
  if constexpr (Geo::TAB_LDS) {
    for (int i = tid; i < P * QT; i += blockDim.x) tws[i] = gtw[i];
    for (int i = tid; i < H; i += blockDim.x) syl[i] = gsy[i];
    __syncthreads();
  }
  if (j < Q) {
    cf w[P];
    static_for<P>([&](auto k1c) {
      constexpr int k1 = decltype(k1c)::value;
      if constexpr (k1 > 0) w[k1] = tw(k1 * QT + j);
    });
    dft<P, -1>(x);
    static_for<P>([&](auto k1c) {
      constexpr int k1 = decltype(k1c)::value;
      ex[k1 * KS + j * S + s] = (k1 == 0) ? x[k1] : cmul(x[k1], w[k1]);
    });
  }
  __syncthreads();
  if (j < P) {  // stage B: lane k1 = j; forward, divide, inverse
    cf y[Q];
    static_for<Q>([&](auto n2c) {
      constexpr int n2 = decltype(n2c)::value;
      y[n2] = ex[j * KS + n2 * S + s];
    });
    dft<Q, -1>(y);
    const float kappa = d.kappa, scale = d.col_scale;
    const float ksx = fmaf(kappa, sxk, 1.0f);
    static_for<Q>([&](auto k2c) {
      constexpr int k2 = decltype(k2c)::value;
      const float den = fmaf(kappa, sy_at(j + P * k2), ksx);
      y[k2] = cscale(y[k2], scale * __builtin_amdgcn_rcpf(den));
    });
    dft<Q, +1>(y);
    // the inverse twiddle of element (k1, n2) (none for n2 = 0): here from
    // the LDS table, else in stage B', where lanes of one k1 read the global
    // table coalesced (the same products either way)
    static_for<Q>([&](auto n2c) {
      constexpr int n2 = decltype(n2c)::value;
      if constexpr (Geo::TAB_LDS)
        ex[j * KS + n2 * S + s] = (n2 == 0) ? y[n2] : cmulc(y[n2], tws[j * QT + n2]);
      else
        ex[j * KS + n2 * S + s] = y[n2];
    });
  }
  __syncthreads();
  if (j < Q) {  // stage B': lane n2 = j, P-point inverse over k1
    if constexpr (Geo::TAB_LDS) {
      static_for<P>([&](auto k1c) {
        constexpr int k1 = decltype(k1c)::value;
        x[k1] = ex[k1 * KS + j * S + s];
      });
    } else {
      cf w[P];
      static_for<P>([&](auto k1c) {
        constexpr int k1 = decltype(k1c)::value;
        w[k1] = cf(gtw[k1 * QT + j]);
      });
      static_for<P>([&](auto k1c) {
        constexpr int k1 = decltype(k1c)::value;
        x[k1] = ex[k1 * KS + j * S + s];
        if (j != 0) x[k1] = cmulc(x[k1], w[k1]);
      });
    }
    dft<P, +1>(x);
    if (col_ok) {
      static_for<P>([&](auto n1c) {
        constexpr int n1 = decltype(n1c)::value;
        out[(size_t)(Q * n1 + j) * ldS] = x[n1];
      });
    }
  }
}

}  // namespace ilsk
