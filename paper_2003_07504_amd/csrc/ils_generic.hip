// Passes for transform lengths without a compiled four-step split: every
// 2/3/5-smooth row length W/2 and column length H up to 4096.
//
// The arithmetic is that of the compiled passes (Algorithm 1 with the
// one-FFT right-hand side of Eq. (9), Sec. 3.2); the transforms are mixed-
// radix Stockham FFTs in LDS whose radix sequence (4s, then a 2, then 3s,
// then 5s) follows from the length at run time, with twiddles from the
// plan's table exp(-2 pi i j / L).  The stencil step, the transform and the
// inverse transform of a row are not fused into one kernel:
//   first  : rhs(u0, f)            -> spectrum (second half spectrum)
//   column : spectrum, in place: forward, divide, inverse
//   middle : c2r(spectrum)         -> u (first half spectrum's memory, as
//                                      real rows of W floats per channel)
//            rhs(u, f)             -> spectrum
//   final  : c2r(spectrum)         -> out
// i.e. 28 bytes per pixel-channel per iteration instead of the fused
// passes' 20.  The scale conventions are those of the compiled passes: the
// row transform leaves a factor 2 and the column pass multiplies by
// 1 / (2 H W).
#include "ils_launch.hpp"

namespace ilsk {

constexpr int kGenThreads = 256;
constexpr int kGenRowMax = 4096;   // complex values per LDS buffer of a row block
constexpr int kGenColCf = 8192;    // complex values per LDS buffer of a column block (H x S)

// One radix-R stage of a Stockham transform of S interleaved sequences of
// length L (element h of sequence s at h * S + s), from src to dst.
// Ns = product of the radices of the earlier stages.
template <int R, int DIR>
__device__ __forceinline__ void stockham_stage(const cf* __restrict__ src, cf* __restrict__ dst, int L, int Ns,
                                               int lgS, const ILS_G cf* __restrict__ tw) {
  const int S = 1 << lgS;
  const int LR = L / R;
  const int step = L / (Ns * R);  // table stride of the twiddle exp(DIR 2 pi i k / (Ns R))
  const int items = LR << lgS;
  for (int it = threadIdx.x; it < items; it += blockDim.x) {
    const int j = it >> lgS;
    const int s = it & (S - 1);
    const int k = j % Ns;
    cf v[R];
    static_for<R>([&](auto qc) {
      constexpr int q = decltype(qc)::value;
      v[q] = src[((j + q * LR) << lgS) + s];
    });
    const int m1 = k * step;
    static_for<R>([&](auto qc) {
      constexpr int q = decltype(qc)::value;
      if constexpr (q > 0) {
        const cf w = cf(tw[q * m1]);
        v[q] = DIR < 0 ? cmul(v[q], w) : cmulc(v[q], w);
      }
    });
    dft<R, DIR>(v);
    const int base = (j - k) * R + k;
    static_for<R>([&](auto qc) {
      constexpr int q = decltype(qc)::value;
      dst[((base + q * Ns) << lgS) + s] = v[q];
    });
  }
}

// L-point DFT (unnormalised, sign DIR) of the S sequences in a; b is the
// second buffer.  Returns the buffer that holds the result in natural order.
// Every thread of the block must call it.
template <int DIR>
__device__ cf* lds_fft(cf* a, cf* b, int L, int lgS, const ILS_G cf* __restrict__ tw) {
  int Ns = 1;
  for (int rem = L; rem > 1;) {
    const int R = (rem % 4 == 0) ? 4 : (rem % 2 == 0) ? 2 : (rem % 3 == 0) ? 3 : 5;
    if (R == 4)
      stockham_stage<4, DIR>(a, b, L, Ns, lgS, tw);
    else if (R == 2)
      stockham_stage<2, DIR>(a, b, L, Ns, lgS, tw);
    else if (R == 3)
      stockham_stage<3, DIR>(a, b, L, Ns, lgS, tw);
    else
      stockham_stage<5, DIR>(a, b, L, Ns, lgS, tw);
    __syncthreads();
    cf* t = a;
    a = b;
    b = t;
    Ns *= R;
    rem /= R;
  }
  return a;
}

__device__ __forceinline__ int wrap(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// Right-hand side row y of one channel, r = f + kappa D^T mu(u) (Eq. (7),
// Eq. (9)), then its R2C transform (x2) into the second half spectrum.
// FROM_A: u is the real image the c2r kernel left in the first half
// spectrum's memory; else u = u0.
template <bool FROM_A, int PEN>
__global__ void __launch_bounds__(kGenThreads) k_gen_rhs(WorkList wl) {
  __shared__ cf buf[2][kGenRowMax];
  int local;
  const FrameDesc d = resolve(wl, blockIdx.x, local);
  const int H = d.H, W = d.W, M = W / 2, ldS = d.ldS;
  const int ch = local / H;
  const int y = local - ch * H;
  const ILS_G float* u = FROM_A ? gm(reinterpret_cast<const float*>(d.specA)) + (size_t)ch * 2 * H * ldS
                                : gm(d.u0) + (size_t)ch * H * W;
  const ILS_G float* uc = u + (size_t)y * W;
  const ILS_G float* uu = u + (size_t)wrap(y - 1, H) * W;
  const ILS_G float* ud = u + (size_t)wrap(y + 1, H) * W;
  const ILS_G float* fr = gm(d.f) + (size_t)ch * H * W + (size_t)y * W;
  const float a_exp = d.a_exp, inv_eps = d.inv_eps, kappa = d.kappa, l2r = d.log2_r;
  auto r_at = [&](int x) {
    const float c = uc[x];
    const float mxl = mu_pen<PEN>(c - uc[wrap(x - 1, W)], a_exp, inv_eps, l2r);
    const float mx0 = mu_pen<PEN>(uc[wrap(x + 1, W)] - c, a_exp, inv_eps, l2r);
    const float myu = mu_pen<PEN>(c - uu[x], a_exp, inv_eps, l2r);
    const float my0 = mu_pen<PEN>(ud[x] - c, a_exp, inv_eps, l2r);
    return fmaf(kappa, (mxl - mx0) + (myu - my0), fr[x]);
  };
  for (int j = threadIdx.x; j < M; j += blockDim.x) buf[0][j] = cf{r_at(2 * j), r_at(2 * j + 1)};
  __syncthreads();
  const cf* Z = lds_fft<-1>(buf[0], buf[1], M, 0, gm(d.tw_row));
  // X'[k] = E - i exp(-i pi k / M) D, E = Z[k] + conj Z[M-k], D = Z[k] - conj Z[M-k]  (= 2 X[k])
  ILS_G cf* X = gm(d.specB) + (size_t)ch * H * ldS + (size_t)y * ldS;
  const ILS_G cf* tw2 = gm(d.tw2_row);
  for (int k = threadIdx.x; k <= M; k += blockDim.x) {
    const cf A = Z[k == M ? 0 : k];
    cf B = Z[k == 0 ? 0 : M - k];
    B.y = -B.y;
    const cf E = cadd(A, B), D = csub(A, B);
    const cf wD = cmul(D, cf(tw2[k]));
    X[k] = cf{E.x + wD.y, E.y - wD.x};
  }
}

// Inverse real transform of row y of the second half spectrum (imaginary
// parts of the DC and Nyquist bins dropped, unnormalised), written as W
// floats: to the first half spectrum's memory (TO_OUT false) or to out,
// blended u + boost (f - u) when boost is non-zero.
template <bool TO_OUT>
__global__ void __launch_bounds__(kGenThreads) k_gen_c2r(WorkList wl) {
  __shared__ cf buf[2][kGenRowMax];
  int local;
  const FrameDesc d = resolve(wl, blockIdx.x, local);
  const int H = d.H, W = d.W, M = W / 2, ldS = d.ldS;
  const int ch = local / H;
  const int y = local - ch * H;
  const ILS_G cf* X = gm(d.specB) + (size_t)ch * H * ldS + (size_t)y * ldS;
  const ILS_G cf* tw2 = gm(d.tw2_row);
  // Z[k] = (X[k] + conj X[M-k]) + i (X[k] - conj X[M-k]) exp(i pi k / M)
  for (int k = threadIdx.x; k < M; k += blockDim.x) {
    cf a = cf(X[k]);
    cf b = cf(X[M - k]);
    if (k == 0) {
      a.y = 0.0f;
      b.y = 0.0f;
    }
    const cf bc = {b.x, -b.y};
    const cf e = cadd(a, bc);
    const cf w = cf(tw2[k]);
    const cf o = cmulc(csub(a, bc), w);
    buf[0][k] = cf{e.x - o.y, e.y + o.x};
  }
  __syncthreads();
  const cf* z = lds_fft<+1>(buf[0], buf[1], M, 0, gm(d.tw_row));
  ILS_G float* dst = TO_OUT ? gm(d.out) + (size_t)ch * H * W + (size_t)y * W
                            : gm(reinterpret_cast<float*>(d.specA)) + (size_t)ch * 2 * H * ldS + (size_t)y * W;
  ILS_G float2* d2 = reinterpret_cast<ILS_G float2*>(dst);
  const float kb = TO_OUT ? d.boost : 0.0f;
  if (kb != 0.0f) {
    const ILS_G float2* f2 = reinterpret_cast<const ILS_G float2*>(gm(d.f) + (size_t)ch * H * W + (size_t)y * W);
    for (int j = threadIdx.x; j < M; j += blockDim.x) {
      const float2 fv = f2[j];
      const cf v = z[j];
      d2[j] = make_float2(fmaf(kb, fv.x - v.x, v.x), fmaf(kb, fv.y - v.y, v.y));
    }
  } else {
    for (int j = threadIdx.x; j < M; j += blockDim.x) d2[j] = make_float2(z[j].x, z[j].y);
  }
}

// Column pass on S columns of the second half spectrum, in place: forward
// column DFT, times 1 / (2 H W (1 + kappa (Sx[k] + Sy[l]))) (Eq. (9)
// denominator), inverse column DFT.  H * S <= kGenColCf.
template <int S>
__global__ void __launch_bounds__(kGenThreads) k_gen_col(WorkList wl) {
  __shared__ cf buf[2][kGenColCf];
  constexpr int lgS = S == 16 ? 4 : S == 8 ? 3 : S == 4 ? 2 : S == 2 ? 1 : 0;
  static_assert((1 << lgS) == S, "S must be a power of two up to 16");
  int local;
  const FrameDesc d = resolve(wl, blockIdx.x, local);
  const int H = d.H, Wh = d.W / 2 + 1, ldS = d.ldS;
  const int nb = (Wh + S - 1) / S;
  const int ch = local / nb;
  const int c0 = (local - ch * nb) * S;
  ILS_G cf* base = gm(d.specB) + (size_t)ch * H * ldS + c0;
  const ILS_G float* sx = gm(d.sx);
  const ILS_G float* sy = gm(d.sy);
  const int n = H << lgS;
  for (int it = threadIdx.x; it < n; it += blockDim.x) {
    const int h = it >> lgS, s = it & (S - 1);
    buf[0][it] = (c0 + s < Wh) ? cf(base[(size_t)h * ldS + s]) : cf{0.0f, 0.0f};
  }
  __syncthreads();
  cf* X = lds_fft<-1>(buf[0], buf[1], H, lgS, gm(d.tw_col));
  cf* other = (X == buf[0]) ? buf[1] : buf[0];
  const float kappa = d.kappa, scale = d.col_scale;
  for (int it = threadIdx.x; it < n; it += blockDim.x) {
    const int l = it >> lgS, s = it & (S - 1);
    const int k = c0 + s < Wh ? c0 + s : Wh - 1;
    const float den = fmaf(kappa, sx[k] + sy[l], 1.0f);
    X[it] = cscale(X[it], scale * __builtin_amdgcn_rcpf(den));
  }
  __syncthreads();
  const cf* Y = lds_fft<+1>(X, other, H, lgS, gm(d.tw_col));
  for (int it = threadIdx.x; it < n; it += blockDim.x) {
    const int h = it >> lgS, s = it & (S - 1);
    if (c0 + s < Wh) base[(size_t)h * ldS + s] = Y[it];
  }
}

hipError_t launch_gen_row(int mode, int pen, const WorkList& wl, hipStream_t st) {
  const dim3 g(wl.total), b(kGenThreads);
  if (mode == ROW_FINAL) {
    hipLaunchKernelGGL((k_gen_c2r<true>), g, b, 0, st, wl);
  } else if (mode == ROW_MID) {
    hipLaunchKernelGGL((k_gen_c2r<false>), g, b, 0, st, wl);
    if (pen == PEN_WELSCH)
      hipLaunchKernelGGL((k_gen_rhs<true, PEN_WELSCH>), g, b, 0, st, wl);
    else
      hipLaunchKernelGGL((k_gen_rhs<true, PEN_CHARBONNIER>), g, b, 0, st, wl);
  } else {
    if (pen == PEN_WELSCH)
      hipLaunchKernelGGL((k_gen_rhs<false, PEN_WELSCH>), g, b, 0, st, wl);
    else
      hipLaunchKernelGGL((k_gen_rhs<false, PEN_CHARBONNIER>), g, b, 0, st, wl);
  }
  return hipGetLastError();
}

template <int S>
hipError_t launch_gen_col(const WorkList& wl, hipStream_t st) {
  hipLaunchKernelGGL((k_gen_col<S>), dim3(wl.total), dim3(kGenThreads), 0, st, wl);
  return hipGetLastError();
}

template <int S>
LenOps make_generic_ops() {
  LenOps o{};
  o.L = 0;
  o.P = 0;
  o.Q = 0;
  o.nrow = 1;
  o.ncol = 1;
  o.row[0] = RowVariant{{1, 1, 1, 1}, kGenThreads, (int)(2 * kGenRowMax * sizeof(cf)), &launch_gen_row};
  o.col[0] = ColVariant{S, kGenThreads, (int)(2 * kGenColCf * sizeof(cf)), &launch_gen_col<S>};
  return o;
}

}  // namespace ilsk

// Launchers of the runtime-length passes for a frame with H rows: one row
// block per (channel, row); column tiles of S = 16, 8, 4 or 2 columns, the
// widest whose H x S values fit one LDS buffer.  H <= 4096.
const ilsk::LenOps* ilsk_generic_ops(int H) {
  static const ilsk::LenOps o16 = ilsk::make_generic_ops<16>();
  static const ilsk::LenOps o8 = ilsk::make_generic_ops<8>();
  static const ilsk::LenOps o4 = ilsk::make_generic_ops<4>();
  static const ilsk::LenOps o2 = ilsk::make_generic_ops<2>();
  if (H * 16 <= ilsk::kGenColCf) return &o16;
  if (H * 8 <= ilsk::kGenColCf) return &o8;
  if (H * 4 <= ilsk::kGenColCf) return &o4;
  return &o2;
}
