// Applications and tooling around the smoother (Sec. 3.4, Sec. 4, Sec. 5):
//   * luminance-only colour mode: Y = 0.299 R + 0.587 G + 0.114 B, smooth Y,
//     add the change of Y back to every channel (a YUV round trip with U, V
//     unchanged);
//   * single- and multi-scale HDR tone mapping on the logarithm of the
//     luminance;
//   * the energy of Eq. (1) for the Charbonnier (Eq. (2)) and Welsch
//     (Eq. (18)) penalties, accumulated in double, for convergence studies.
// Elementwise kernels are grid-stride loops over the pixels of a plane.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <vector>

#include "../../include/ils.h"

namespace {

constexpr int kThreads = 256;
constexpr int kEnergyBlocks = 256;

__global__ void __launch_bounds__(kThreads) k_luma(const float* __restrict__ rgb, float* __restrict__ y, long long plane) {
  const long long stride = (long long)gridDim.x * kThreads;
  for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < plane; i += stride)
    y[i] = fmaf(0.114f, rgb[i + 2 * plane], fmaf(0.587f, rgb[i + plane], 0.299f * rgb[i]));
}

// out_c = f_c + (v - Y) for c = 0, 1, 2
__global__ void __launch_bounds__(kThreads) k_recombine(const float* f, const float* __restrict__ y,
                                                         const float* __restrict__ v, float* out, long long plane) {
  const long long stride = (long long)gridDim.x * kThreads;
  for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < plane; i += stride) {
    const float dlt = v[i] - y[i];
    const float r = f[i], g = f[i + plane], b = f[i + 2 * plane];
    out[i] = r + dlt;
    out[i + plane] = g + dlt;
    out[i + 2 * plane] = b + dlt;
  }
}

// log of the luminance, floored (HDR tone mapping works on log Y)
__global__ void __launch_bounds__(kThreads) k_loglum(const float* __restrict__ rgb, float* __restrict__ L,
                                                      long long plane, float floor_y) {
  const long long stride = (long long)gridDim.x * kThreads;
  for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < plane; i += stride) {
    const float y = fmaf(0.114f, rgb[i + 2 * plane], fmaf(0.587f, rgb[i + plane], 0.299f * rgb[i]));
    L[i] = logf(fmaxf(y, floor_y));
  }
}

// min and max of a plane: per-block partials, then one block
constexpr int kMinMaxBlocks = 256;
__global__ void __launch_bounds__(kThreads) k_minmax_partial(const float* __restrict__ b, long long plane,
                                                              float* partial) {
  float lo = INFINITY, hi = -INFINITY;
  for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < plane; i += (long long)kMinMaxBlocks * kThreads) {
    const float v = b[i];
    lo = fminf(lo, v);
    hi = fmaxf(hi, v);
  }
  __shared__ float rl[kThreads], rh[kThreads];
  rl[threadIdx.x] = lo;
  rh[threadIdx.x] = hi;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      rl[threadIdx.x] = fminf(rl[threadIdx.x], rl[threadIdx.x + s]);
      rh[threadIdx.x] = fmaxf(rh[threadIdx.x], rh[threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = rl[0];
    partial[2 * blockIdx.x + 1] = rh[0];
  }
}

__global__ void __launch_bounds__(kMinMaxBlocks) k_minmax_final(const float* partial, float* mm) {
  __shared__ float rl[kMinMaxBlocks], rh[kMinMaxBlocks];
  rl[threadIdx.x] = partial[2 * threadIdx.x];
  rh[threadIdx.x] = partial[2 * threadIdx.x + 1];
  __syncthreads();
  for (int s = kMinMaxBlocks / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      rl[threadIdx.x] = fminf(rl[threadIdx.x], rl[threadIdx.x + s]);
      rh[threadIdx.x] = fmaxf(rh[threadIdx.x], rh[threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    mm[0] = rl[0];
    mm[1] = rh[0];
  }
}

// out_c = f_c exp(L' - L), L' = (B - max B) s + detail (L - B), s = log(contrast) / (max B - min B)
__global__ void __launch_bounds__(kThreads) k_tonemap(const float* f, const float* __restrict__ L,
                                                       const float* __restrict__ B, const float* __restrict__ mm,
                                                       float log_contrast, float detail, float* out, long long plane) {
  const float bmin = mm[0], bmax = mm[1];
  const float s = bmax > bmin ? log_contrast / (bmax - bmin) : 1.0f;
  const long long stride = (long long)gridDim.x * kThreads;
  for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < plane; i += stride) {
    const float l = L[i], b = B[i];
    const float g = expf(fmaf(b - bmax, s, detail * (l - b)) - l);
    const float r = f[i], gg = f[i + plane], bb = f[i + 2 * plane];
    out[i] = r * g;
    out[i + plane] = gg * g;
    out[i + 2 * plane] = bb * g;
  }
}

// Multi-scale version: K smoothed levels B_1..B_K of L (increasing lambda),
// detail layers D_1 = L - B_1, D_i = B_{i-1} - B_i kept times w_i, base B_K
// compressed as in k_tonemap (mm = its min and max).
constexpr int kMaxScales = 4;
struct MultiScaleArgs {
  const float* B[kMaxScales];
  float w[kMaxScales];
  int K;
};
__global__ void __launch_bounds__(kThreads) k_tonemap_ms(const float* f, const float* __restrict__ L, MultiScaleArgs a,
                                                          const float* __restrict__ mm, float log_contrast, float* out,
                                                          long long plane) {
  const float bmin = mm[0], bmax = mm[1];
  const float s = bmax > bmin ? log_contrast / (bmax - bmin) : 1.0f;
  const long long stride = (long long)gridDim.x * kThreads;
  for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < plane; i += stride) {
    const float l = L[i];
    float prev = l, acc = 0.0f;
    for (int k = 0; k < a.K; ++k) {
      const float b = a.B[k][i];
      acc = fmaf(a.w[k], prev - b, acc);
      prev = b;
    }
    const float g = expf(fmaf(prev - bmax, s, acc) - l);
    const float r = f[i], gg = f[i + plane], bb = f[i + 2 * plane];
    out[i] = r * g;
    out[i + plane] = gg * g;
    out[i + 2 * plane] = bb * g;
  }
}

struct EnergyArgs {
  const float* f;
  const float* u;
  int H, W, C;
  int penalty;
  double lambda, half_p, eps, inv_2g2, two_g2;
};

__device__ __forceinline__ double phi(const EnergyArgs& a, double x) {
  if (a.penalty == ILS_PENALTY_WELSCH) return a.two_g2 * (1.0 - exp(-x * x * a.inv_2g2));  // Eq. (18)
  return pow(x * x + a.eps, a.half_p);                                                  // Eq. (2)
}

// Per-block partial sums of (u - f)^2 + lambda (phi(D_x u) + phi(D_y u)),
// periodic differences, in double.  Blocks stride over image rows (all
// channels), threads over the columns of a row.
__global__ void __launch_bounds__(kThreads) k_energy_partial(EnergyArgs a, double* partial) {
  const long long plane = (long long)a.H * a.W;
  double acc = 0.0;
  for (int row = blockIdx.x; row < a.C * a.H; row += kEnergyBlocks) {
    const int ch = row / a.H, y = row - ch * a.H;
    const int yd = y + 1 == a.H ? 0 : y + 1;
    const float* uc = a.u + (long long)ch * plane;
    const float* ur = uc + (long long)y * a.W;
    const float* ud = uc + (long long)yd * a.W;
    const float* fr = a.f + (long long)ch * plane + (long long)y * a.W;
    for (int x = threadIdx.x; x < a.W; x += kThreads) {
      const int xr = x + 1 == a.W ? 0 : x + 1;
      const double u0 = ur[x];
      const double d = u0 - (double)fr[x];
      acc += d * d + a.lambda * (phi(a, (double)ur[xr] - u0) + phi(a, (double)ud[x] - u0));
    }
  }
  __shared__ double red[kThreads];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(kEnergyBlocks) k_energy_final(const double* partial, double* energy) {
  __shared__ double red[kEnergyBlocks];
  red[threadIdx.x] = partial[threadIdx.x];
  __syncthreads();
  for (int s = kEnergyBlocks / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) *energy = red[0];
}

int grid_for(long long n) {
  long long g = (n + kThreads - 1) / kThreads;
  return (int)(g < 2048 ? (g < 1 ? 1 : g) : 2048);
}

}  // namespace

extern "C++" int ilsk_plan_scratch(ils_plan* plan, void** scratch, size_t* bytes, void** stream);

// Launchers used by the planner (same stream as the plan).
hipError_t ilsk_launch_luma(const float* rgb, float* y, long long plane, hipStream_t st) {
  hipLaunchKernelGGL(k_luma, dim3(grid_for(plane)), dim3(kThreads), 0, st, rgb, y, plane);
  return hipGetLastError();
}

hipError_t ilsk_launch_recombine(const float* f, const float* y, const float* v, float* out, long long plane,
                                 hipStream_t st) {
  hipLaunchKernelGGL(k_recombine, dim3(grid_for(plane)), dim3(kThreads), 0, st, f, y, v, out, plane);
  return hipGetLastError();
}

hipError_t ilsk_launch_loglum(const float* rgb, float* L, long long plane, float floor_y, hipStream_t st) {
  hipLaunchKernelGGL(k_loglum, dim3(grid_for(plane)), dim3(kThreads), 0, st, rgb, L, plane, floor_y);
  return hipGetLastError();
}

// min/max of B into mm[0..1]; scratch holds 2 * 256 floats of partials
hipError_t ilsk_launch_minmax(const float* B, long long plane, float* scratch, float* mm, hipStream_t st) {
  hipLaunchKernelGGL(k_minmax_partial, dim3(kMinMaxBlocks), dim3(kThreads), 0, st, B, plane, scratch);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_minmax_final, dim3(1), dim3(kMinMaxBlocks), 0, st, scratch, mm);
  return hipGetLastError();
}

hipError_t ilsk_launch_tonemap(const float* f, const float* L, const float* B, const float* mm, float log_contrast,
                               float detail, float* out, long long plane, hipStream_t st) {
  hipLaunchKernelGGL(k_tonemap, dim3(grid_for(plane)), dim3(kThreads), 0, st, f, L, B, mm, log_contrast, detail, out,
                     plane);
  return hipGetLastError();
}

hipError_t ilsk_launch_tonemap_ms(const float* f, const float* L, const float* const* B, const float* w, int K,
                                  const float* mm, float log_contrast, float* out, long long plane, hipStream_t st) {
  if (K < 1 || K > kMaxScales) return hipErrorInvalidValue;
  MultiScaleArgs a{};
  for (int k = 0; k < K; ++k) {
    a.B[k] = B[k];
    a.w[k] = w[k];
  }
  a.K = K;
  hipLaunchKernelGGL(k_tonemap_ms, dim3(grid_for(plane)), dim3(kThreads), 0, st, f, L, a, mm, log_contrast, out, plane);
  return hipGetLastError();
}

static int energy_impl(ils_plan* plan, const float* f, const float* u, int H, int W, int C, float lambda,
                       int penalty, float p, float eps, float gamma, double* energy) {
  if (!plan || !f || !u || !energy || H < 2 || W < 2 || C < 1) return ILS_ERR_INVALID_ARG;
  if (!std::isfinite(lambda) || lambda < 0.0f) return ILS_ERR_INVALID_ARG;
  EnergyArgs a{};
  a.f = f;
  a.u = u;
  a.H = H;
  a.W = W;
  a.C = C;
  a.penalty = penalty;
  a.lambda = lambda;
  if (penalty == ILS_PENALTY_WELSCH) {
    if (!std::isfinite(gamma) || !(gamma > 0.0f)) return ILS_ERR_INVALID_ARG;
    a.two_g2 = 2.0 * (double)gamma * (double)gamma;
    a.inv_2g2 = 1.0 / a.two_g2;
  } else {
    if (!std::isfinite(p) || !(p > 0.0f) || p > 2.0f || !std::isfinite(eps) || !(eps > 0.0f))
      return ILS_ERR_INVALID_ARG;
    a.half_p = (double)p / 2.0;
    a.eps = eps;
  }
  void* scratch = nullptr;
  size_t bytes = 0;
  void* stream = nullptr;
  if (ilsk_plan_scratch(plan, &scratch, &bytes, &stream) != ILS_OK) return ILS_ERR_INVALID_ARG;
  if (bytes < kEnergyBlocks * sizeof(double)) return ILS_ERR_WORKSPACE;
  double* partial = static_cast<double*>(scratch);
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(k_energy_partial, dim3(kEnergyBlocks), dim3(kThreads), 0, st, a, partial);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(kEnergyBlocks), 0, st, partial, energy);
    e = hipGetLastError();
  }
  return e == hipSuccess ? ILS_OK : ILS_ERR_HIP;
}

extern "C" int ils_energy(ils_plan* plan, const float* f, const float* u, int H, int W, int C, float lambda,
                          float p, float eps, double* energy) {
  return energy_impl(plan, f, u, H, W, C, lambda, ILS_PENALTY_CHARBONNIER, p, eps, 0.0f, energy);
}

extern "C" int ils_energy_welsch(ils_plan* plan, const float* f, const float* u, int H, int W, int C,
                                 float lambda, float gamma, double* energy) {
  return energy_impl(plan, f, u, H, W, C, lambda, ILS_PENALTY_WELSCH, 0.0f, 0.0f, gamma, energy);
}
