// Per-frame RMS difference (fixed-point residual of a candidate output:
// rms(T(v) - v) over all pixels and channels of a frame).  Deterministic two
// level reduction in double: fixed-size per-block partials, then one block
// per frame sums its partials in a fixed order.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <vector>

#include "../../include/ils.h"

namespace {

constexpr int kThreads = 256;
constexpr int kBlocksPerFrame = 128;
constexpr int kMaxFrames = 512;

struct RmsJob {
  const float* a;
  const float* b;
  long long count;
};

__global__ void __launch_bounds__(kThreads) k_rms_partial(const RmsJob* jobs, double* partial) {
  const int frame = blockIdx.y;
  const RmsJob j = jobs[frame];
  double acc = 0.0;
  const long long stride = (long long)kBlocksPerFrame * kThreads;
  for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < j.count; i += stride) {
    double d = (double)j.a[i] - (double)j.b[i];
    acc += d * d;
  }
  __shared__ double red[kThreads];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[(size_t)frame * kBlocksPerFrame + blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(kBlocksPerFrame) k_rms_final(const RmsJob* jobs, const double* partial,
                                                               float* rms) {
  const int frame = blockIdx.x;
  __shared__ double red[kBlocksPerFrame];
  red[threadIdx.x] = partial[(size_t)frame * kBlocksPerFrame + threadIdx.x];
  __syncthreads();
  for (int s = kBlocksPerFrame / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const long long c = jobs[frame].count;
    rms[frame] = c > 0 ? (float)sqrt(red[0] / (double)c) : 0.0f;
  }
}

}  // namespace

// Scratch for the reduction lives in the plan workspace's header area; the
// accessor is defined next to the plan.
extern "C++" int ilsk_plan_scratch(ils_plan* plan, void** scratch, size_t* bytes, void** stream);
extern "C++" int ilsk_plan_upload(ils_plan* plan, void* dst, const void* src, size_t bytes);

extern "C" int ils_rms_diff(ils_plan* plan, const float* const* a, const float* const* b,
                            const long long* count, int n, float* rms) {
  if (!plan || !a || !b || !count || !rms || n < 1 || n > kMaxFrames) return ILS_ERR_INVALID_ARG;
  for (int i = 0; i < n; ++i)
    if (!a[i] || !b[i] || count[i] < 0) return ILS_ERR_INVALID_ARG;
  void* scratch = nullptr;
  size_t bytes = 0;
  void* stream = nullptr;
  if (ilsk_plan_scratch(plan, &scratch, &bytes, &stream) != ILS_OK) return ILS_ERR_INVALID_ARG;
  const size_t jobs_bytes = ((size_t)n * sizeof(RmsJob) + 255) / 256 * 256;
  const size_t part_bytes = (size_t)n * kBlocksPerFrame * sizeof(double);
  if (jobs_bytes + part_bytes > bytes) return ILS_ERR_WORKSPACE;
  std::vector<RmsJob> jobs(n);
  for (int i = 0; i < n; ++i) jobs[i] = RmsJob{a[i], b[i], count[i]};
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(scratch);
  RmsJob* djobs = reinterpret_cast<RmsJob*>(base);
  double* partial = reinterpret_cast<double*>(base + jobs_bytes);
  if (ilsk_plan_upload(plan, djobs, jobs.data(), n * sizeof(RmsJob)) != ILS_OK) return ILS_ERR_HIP;
  hipError_t e = hipSuccess;
  {
    hipLaunchKernelGGL(k_rms_partial, dim3(kBlocksPerFrame, n), dim3(kThreads), 0, st, djobs, partial);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_rms_final, dim3(n), dim3(kBlocksPerFrame), 0, st, djobs, partial, rms);
    e = hipGetLastError();
  }
  return e == hipSuccess ? ILS_OK : ILS_ERR_HIP;
}
