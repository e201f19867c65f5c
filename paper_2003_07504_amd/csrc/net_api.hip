// Learned surrogate of the ILS output: training and inference kernels plus
// the C ABI declared in include/ils_net.h, and the residual-gated inference
// that falls back to plain ILS.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/ils.h"
#include "../../include/ils_net.h"
#include "net_kernels.hpp"

// The stream a plan currently enqueues on (library-internal, ils_api.cpp).
void* ilsk_plan_stream(ils_plan* plan);

using namespace ilsn;

namespace {

// ---------------------------------------------------------------- network
struct Layer {
  int ci, co;    // real channels
  int cip, cop;  // padded channels of the forward convolution
  int w_off, b_off;  // offsets (floats) in the master parameter array
};

// Layer i: 5 -> 32, four times 32 -> 32, 32 -> 3.  Parameters are stored
// layer by layer as w[co][ci][3][3] followed by b[co].
__host__ __device__ constexpr Layer layer_def(int i) {
  int off = 0;
  Layer L{0, 0, 0, 0, 0, 0};
  for (int k = 0; k <= i; ++k) {
    const int ci = (k == 0) ? 5 : 32, co = (k == 5) ? 3 : 32;
    L = Layer{ci, co, ci == 5 ? 8 : 32, co == 3 ? 16 : 32, off, off + co * ci * 9};
    off += co * ci * 9 + co;
  }
  return L;
}

struct Net {
  Layer L[6];
  size_t nparams;
  Net() {
    for (int i = 0; i < 6; ++i) L[i] = layer_def(i);
    nparams = (size_t)L[5].b_off + L[5].co;
  }
};
const Net kNet;

// channels of the gradient tensor flowing into the output of layer i
inline int gchan(int i) { return kNet.L[i].co == 3 ? 8 : 32; }

inline size_t al(size_t v) { return (v + 255) / 256 * 256; }

constexpr int kWgradBlocks = 256;
constexpr int kLossBlocks = 256;

// --------------------------------------------------------- small kernels
// dst[0] = a, dst[1] = b (a frame's lambda and p for the input maps)
__global__ void k_set_pair(float* dst, float a, float b) {
  if (threadIdx.x == 0) {
    dst[0] = a;
    dst[1] = b;
  }
}

__global__ void __launch_bounds__(256) k_pack_input(const float* f, const float* lam, const float* p, bf16* x0,
                                                   int B, int H, int W) {
  const size_t plane = (size_t)H * W;
  const size_t n = (size_t)B * plane;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
    const size_t img = i / plane, pix = i - img * plane;
    const float* fi = f + img * 3 * plane + pix;
    bf16 o[8];
    o[0] = f2bf(fi[0]);
    o[1] = f2bf(fi[plane]);
    o[2] = f2bf(fi[2 * plane]);
    o[3] = f2bf(lam[img]);
    o[4] = f2bf(p[img]);
    o[5] = o[6] = o[7] = f2bf(0.0f);
    *reinterpret_cast<uint4*>(&x0[i * 8]) = *reinterpret_cast<const uint4*>(o);
  }
}

// g6 = d(mean squared error)/dv = 2 (v - t) / n, NHWC bf16 (8 channels);
// per-block partial sums of (v - t)^2 in double.
__global__ void __launch_bounds__(256) k_loss_grad(const float* v, const float* t, bf16* g, double* partial,
                                                  int B, int H, int W) {
  const size_t plane = (size_t)H * W;
  const size_t n = (size_t)B * plane;
  const float scale = (float)(2.0 / (3.0 * (double)n));
  double acc = 0.0;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
    const size_t img = i / plane, pix = i - img * plane;
    const size_t base = img * 3 * plane + pix;
    bf16 o[8];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float d = v[base + c * plane] - t[base + c * plane];
      acc += (double)d * d;
      o[c] = f2bf(scale * d);
    }
    o[3] = o[4] = o[5] = o[6] = o[7] = f2bf(0.0f);
    *reinterpret_cast<uint4*>(&g[i * 8]) = *reinterpret_cast<const uint4*>(o);
  }
  __shared__ double red[256];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void k_loss_final(const double* partial, int nb, double n, float* loss) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < nb; ++i) s += partial[i];
    *loss = (float)(s / n);
  }
}

// Partial weight and bias gradients of one convolution on the MFMA units:
//   dW[co][ci][tap] = sum_pixels g[pixel][co] x[pixel + shift(tap)][ci]
// is, for each tap, D[co][ci] += sum_k G[co][k] X_tap[k][ci] with k running
// over the 32 pixels of one tile row (one K block of v_mfma_f32_16x16x32_bf16).
// The (16-row co block, 16-column ci block) pairs are dealt to the four
// waves; when there are two pairs (first and last layers), two waves share a
// pair, taking alternate tile rows, and add up through LDS at the end.  The
// fragments are gathered from the NHWC tiles in LDS (channels beyond the
// layer's read as zero).  db[co] = sum g[pixel][co] on the VALU.  Blocks
// stride over TH x TW pixel tiles and write one partial row each (reduced
// in a fixed order afterwards: deterministic).
template <int GC, int XC>
__global__ void __launch_bounds__(256) k_wgrad_mfma(const bf16* g, const bf16* x, float* partial, int gcr, int xcr,
                                                   int B, int H, int W) {
  constexpr int LH = TH + 2, LW = TW + 2;
  constexpr int MB = (GC + 15) / 16, NB = (XC + 15) / 16;
  constexpr int PAIRS = MB * NB;  // 2 or 4
  constexpr int RG = 4 / PAIRS;   // waves per pair
  static_assert(PAIRS * RG == 4, "four waves per block");
  constexpr int G_BYTES = TH * TW * GC * 2, X_BYTES = LH * LW * XC * 2;
  constexpr int RED_BYTES = 2 * 64 * 36 * 4;  // accumulators of two waves
  constexpr int LDS_BYTES = (G_BYTES + X_BYTES) > RED_BYTES ? (G_BYTES + X_BYTES) : RED_BYTES;
  __shared__ __attribute__((aligned(16))) unsigned char lds[LDS_BYTES];
  __shared__ float bred[256];
  bf16* gt = reinterpret_cast<bf16*>(lds);
  bf16* xt = reinterpret_cast<bf16*>(lds + G_BYTES);
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int pair = wave % PAIRS, rg = wave / PAIRS;
  const int mb = pair / NB, nb = pair - mb * NB;
  const int m = lane & 15, kc = lane >> 4;
  const int co_a = mb * 16 + m;   // A row of this lane
  const int ci_b = nb * 16 + m;   // B column of this lane
  f32x4 acc[9];
#pragma unroll
  for (int tap = 0; tap < 9; ++tap) acc[tap] = f32x4{0.f, 0.f, 0.f, 0.f};
  float accb = 0.0f;
  const int bco = tid % GC;  // bias: channel and pixel phase of this thread
  const int bph = tid / GC;

  const int tiles_x = (W + TW - 1) / TW, tiles_y = (H + TH - 1) / TH;
  const int ntiles = B * tiles_x * tiles_y;
  const size_t plane = (size_t)H * W;
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int img = tile / (tiles_x * tiles_y);
    const int rem = tile - img * tiles_x * tiles_y;
    const int ty = rem / tiles_x, tx = rem - ty * tiles_x;
    const int y0 = ty * TH, x0 = tx * TW;
    for (int i = tid; i < TH * TW * (GC / 8); i += 256) {
      const int pix = i / (GC / 8), chn = i - pix * (GC / 8);
      const int py = pix / TW, px = pix - py * TW;
      const int gy = y0 + py, gx = x0 + px;
      uint4 v = make_uint4(0, 0, 0, 0);
      if (gy < H && gx < W) v = *reinterpret_cast<const uint4*>(&g[((size_t)img * plane + (size_t)gy * W + gx) * GC + chn * 8]);
      *reinterpret_cast<uint4*>(&gt[pix * GC + chn * 8]) = v;
    }
    for (int i = tid; i < LH * LW * (XC / 8); i += 256) {
      const int pix = i / (XC / 8), chn = i - pix * (XC / 8);
      const int ly = pix / LW, lx = pix - ly * LW;
      const int gy = wrapi(y0 + ly - 1, H), gx = wrapi(x0 + lx - 1, W);
      *reinterpret_cast<uint4*>(&xt[pix * XC + chn * 8]) =
          *reinterpret_cast<const uint4*>(&x[((size_t)img * plane + (size_t)gy * W + gx) * XC + chn * 8]);
    }
    __syncthreads();
    for (int p = bph; p < TH * TW; p += 256 / GC) accb += bf2f(gt[p * GC + bco]);
    for (int py = rg; py < TH; py += RG) {
      bf16x8 a;
#pragma unroll
      for (int e = 0; e < 8; ++e) a[e] = co_a < GC ? gt[(py * TW + kc * 8 + e) * GC + co_a] : f2bf(0.0f);
#pragma unroll
      for (int tap = 0; tap < 9; ++tap) {
        const int ta = tap / 3, tc = tap - 3 * ta;
        bf16x8 b;
#pragma unroll
        for (int e = 0; e < 8; ++e)
          b[e] = ci_b < XC ? xt[((py + ta) * LW + kc * 8 + e + tc) * XC + ci_b] : f2bf(0.0f);
        acc[tap] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[tap], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  // waves of the second row group hand their sums to the first
  float* red = reinterpret_cast<float*>(lds);
  if (RG == 2 && rg == 1) {
#pragma unroll
    for (int tap = 0; tap < 9; ++tap)
#pragma unroll
      for (int i = 0; i < 4; ++i) red[((pair * 9 + tap) * 4 + i) * 64 + lane] = acc[tap][i];
  }
  bred[tid] = accb;
  __syncthreads();
  float* out = partial + (size_t)blockIdx.x * (size_t)(gcr * xcr * 9 + gcr);
  if (rg == 0) {
    const int ci = nb * 16 + m;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int co = mb * 16 + 4 * kc + i;
      if (co >= gcr || ci >= xcr) continue;
#pragma unroll
      for (int tap = 0; tap < 9; ++tap) {
        float v = acc[tap][i];
        if (RG == 2) v += red[((pair * 9 + tap) * 4 + i) * 64 + lane];
        out[((size_t)co * xcr + ci) * 9 + tap] = v;
      }
    }
  }
  if (tid < gcr) {
    float sb = 0.0f;
    for (int j = 0; j < 256 / GC; ++j) sb += bred[j * GC + tid];
    out[(size_t)gcr * xcr * 9 + tid] = sb;
  }
}

// grad[k] = sum over blocks (fixed order) of partial[b][k]
__global__ void __launch_bounds__(256) k_reduce_partials(const float* partial, int nblocks, int len, float* grad) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= len) return;
  double s = 0.0;
  for (int b = 0; b < nblocks; ++b) s += partial[(size_t)b * len + k];
  grad[k] = (float)s;
}

// Adam with bias correction (Kingma & Ba): fp32 master parameters.
__global__ void __launch_bounds__(256) k_adam(float* prm, float* m, float* v, const float* g, int n, float lr,
                                             float b1, float b2, float eps, float c1, float c2) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float mhat = mi / c1, vhat = vi / c2;
  prm[i] -= lr * mhat / (sqrtf(vhat) + eps);
}

// Pack master fp32 weights into the bf16 fragment layouts.
//   forward WF[co][tap*CIP + ci]    = w[co][ci][tap]
//   dgrad   WD[ci][tap'*COPg + co]  = w[co][ci][8 - tap']   (flipped, transposed)
// and the padded fp32 biases.
struct PackArgs {
  const float* master;
  bf16* wf[6];
  bf16* wd[6];
  float* bias[6];
};

__global__ void __launch_bounds__(256) k_pack_weights(PackArgs a) {
  const int layer = blockIdx.y;
  const Layer L = layer_def(layer);
  const float* w = a.master + L.w_off;
  const float* b = a.master + L.b_off;
  const int kpf = kpad(L.cip);
  const int nf = L.cop * kpf;
  const int gcp = (L.co == 3) ? 8 : 32;  // channels of the gradient tensor
  const int kpd = kpad(gcp);
  const int nd = 32 * kpd;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < nf + nd + L.cop; i += gridDim.x * 256) {
    if (i < nf) {
      const int co = i / kpf, k = i - co * kpf;
      const int tap = k / L.cip, ci = k - tap * L.cip;
      float val = 0.0f;
      if (co < L.co && ci < L.ci && tap < 9) val = w[((size_t)co * L.ci + ci) * 9 + tap];
      a.wf[layer][i] = f2bf(val);
    } else if (i < nf + nd) {
      if (layer == 0) continue;  // the image gradient is never needed
      const int j = i - nf;
      const int ci = j / kpd, k = j - ci * kpd;
      const int tapd = k / gcp, co = k - tapd * gcp;
      float val = 0.0f;
      if (co < L.co && ci < L.ci && tapd < 9) val = w[((size_t)co * L.ci + ci) * 9 + (8 - tapd)];
      a.wd[layer][j] = f2bf(val);
    } else {
      const int co = i - nf - nd;
      a.bias[layer][co] = co < L.co ? b[co] : 0.0f;
    }
  }
}

}  // namespace

// ------------------------------------------------------------------ state
struct ils_net {
  int max_B, max_H, max_W;
  hipStream_t stream;
  char* ws;
  size_t ws_bytes;
  int last_error;
  long long step;
  // device buffers (carved from the workspace)
  float* master;
  float* adam_m;
  float* adam_v;
  float* grad;
  bf16* wf[6];
  bf16* wd[6];
  float* bias[6];
  bf16* act[6];   // act[0] = x0 (8 ch), act[1..5] = a1..a5 (32 ch)
  bf16* gbuf[2];  // gradient ping-pong (32 ch)
  float* zbuf;    // v (B, 3, H, W) scratch
  float* partial; // wgrad partials
  double* lpart;  // loss partials
  float* loss;
};

namespace {

size_t net_layout(int B, int H, int W, ils_net* n) {
  const size_t px = (size_t)B * H * W;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = al(off + bytes);
    return o;
  };
  size_t o_master = take(kNet.nparams * 4), o_m = take(kNet.nparams * 4), o_v = take(kNet.nparams * 4),
         o_g = take(kNet.nparams * 4);
  size_t o_wf[6], o_wd[6], o_b[6];
  for (int i = 0; i < 6; ++i) {
    o_wf[i] = take((size_t)kNet.L[i].cop * kpad(kNet.L[i].cip) * 2);
    o_wd[i] = take((size_t)32 * kpad(gchan(i)) * 2);
    o_b[i] = take((size_t)kNet.L[i].cop * 4);
  }
  size_t o_act[6];
  o_act[0] = take(px * 8 * 2);
  for (int i = 1; i < 6; ++i) o_act[i] = take(px * 32 * 2);
  size_t o_gb0 = take(px * 32 * 2), o_gb1 = take(px * 32 * 2);
  size_t o_z = take(px * 3 * 4);
  size_t o_part = take((size_t)kWgradBlocks * (32 * 32 * 9 + 32) * 4);
  size_t o_lp = take(kLossBlocks * 8);
  size_t o_loss = take(4);
  if (n) {
    char* b = n->ws;
    n->master = (float*)(b + o_master);
    n->adam_m = (float*)(b + o_m);
    n->adam_v = (float*)(b + o_v);
    n->grad = (float*)(b + o_g);
    for (int i = 0; i < 6; ++i) {
      n->wf[i] = (bf16*)(b + o_wf[i]);
      n->wd[i] = (bf16*)(b + o_wd[i]);
      n->bias[i] = (float*)(b + o_b[i]);
      n->act[i] = (bf16*)(b + o_act[i]);
    }
    n->gbuf[0] = (bf16*)(b + o_gb0);
    n->gbuf[1] = (bf16*)(b + o_gb1);
    n->zbuf = (float*)(b + o_z);
    n->partial = (float*)(b + o_part);
    n->lpart = (double*)(b + o_lp);
    n->loss = (float*)(b + o_loss);
  }
  return off;
}

int rec(ils_net* n, hipError_t e) {
  if (e == hipSuccess) return ILS_OK;
  if (n && n->last_error == ILS_OK) n->last_error = (int)e;
  return ILS_ERR_HIP;
}

// Workgroups of `kernel` the current device holds at once (the convolution
// kernels loop over tiles, so a larger grid only adds weight reloads).
int resident_blocks(const void* kernel) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 1024;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) return 1024;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, NTHREADS, 0) != hipSuccess || per_cu <= 0)
    per_cu = 1;
  return cus * per_cu;
}

int conv_grid(long long tiles, int cap) { return (int)(tiles < cap ? tiles : cap); }

template <int CIP, int COP, int MODE>
hipError_t conv(const ConvArgs& a, hipStream_t st) {
  static const int cap_near = resident_blocks(reinterpret_cast<const void*>(&k_conv<CIP, COP, MODE, true>));
  static const int cap_any = resident_blocks(reinterpret_cast<const void*>(&k_conv<CIP, COP, MODE, false>));
  const long long tiles = (long long)a.B * ((a.H + TH - 1) / TH) * ((a.W + TW - 1) / TW);
  if (a.H >= TH + 2 && a.W >= TW + 2)
    hipLaunchKernelGGL((k_conv<CIP, COP, MODE, true>), dim3(conv_grid(tiles, cap_near)), dim3(NTHREADS), 0, st, a);
  else
    hipLaunchKernelGGL((k_conv<CIP, COP, MODE, false>), dim3(conv_grid(tiles, cap_any)), dim3(NTHREADS), 0, st, a);
  return hipGetLastError();
}

// forward through the six layers; v written to `v` (planar fp32)
hipError_t run_forward(ils_net* n, const float* f, const float* lam, const float* p, int B, int H, int W, float* v) {
  hipStream_t st = n->stream;
  const size_t px = (size_t)B * H * W;
  int blocks = (int)((px + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_pack_input, dim3(blocks), dim3(256), 0, st, f, lam, p, n->act[0], B, H, W);
  hipError_t e = hipGetLastError();
  for (int i = 0; i < 6 && e == hipSuccess; ++i) {
    ConvArgs a{};
    a.in = n->act[i];
    a.wfrag = n->wf[i];
    a.bias = n->bias[i];
    a.B = B;
    a.H = H;
    a.W = W;
    if (i == 0) {
      a.out = n->act[1];
      e = conv<8, 32, CONV_RELU>(a, st);
    } else if (i < 5) {
      a.out = n->act[i + 1];
      e = conv<32, 32, CONV_RELU>(a, st);
    } else {
      a.f = f;
      a.v = v;
      e = conv<32, 16, CONV_LAST>(a, st);
    }
  }
  return e;
}

// gradients of the loss for the batch whose forward pass is in n->act / zbuf
hipError_t run_backward(ils_net* n, const float* t, int B, int H, int W) {
  hipStream_t st = n->stream;
  const size_t px = (size_t)B * H * W;
  hipLaunchKernelGGL(k_loss_grad, dim3(kLossBlocks), dim3(256), 0, st, n->zbuf, t, n->gbuf[0], n->lpart, B, H, W);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(64), 0, st, n->lpart, kLossBlocks, 3.0 * (double)px, n->loss);
  e = hipGetLastError();
  int cur = 0;
  for (int i = 5; i >= 0 && e == hipSuccess; --i) {
    const Layer& L = kNet.L[i];
    const bf16* g = n->gbuf[cur];
    const bf16* x = n->act[i];
    const int len = L.co * L.ci * 9 + L.co;
    if (i == 5)
      hipLaunchKernelGGL((k_wgrad_mfma<8, 32>), dim3(kWgradBlocks), dim3(256), 0, st, g, x, n->partial, L.co, L.ci, B,
                         H, W);
    else if (i == 0)
      hipLaunchKernelGGL((k_wgrad_mfma<32, 8>), dim3(kWgradBlocks), dim3(256), 0, st, g, x, n->partial, L.co, L.ci, B,
                         H, W);
    else
      hipLaunchKernelGGL((k_wgrad_mfma<32, 32>), dim3(kWgradBlocks), dim3(256), 0, st, g, x, n->partial, L.co, L.ci,
                         B, H, W);
    e = hipGetLastError();
    if (e != hipSuccess) break;
    hipLaunchKernelGGL(k_reduce_partials, dim3((len + 255) / 256), dim3(256), 0, st, n->partial, kWgradBlocks, len,
                       n->grad + L.w_off);
    e = hipGetLastError();
    if (e != hipSuccess || i == 0) break;
    ConvArgs a{};
    a.in = g;
    a.wfrag = n->wd[i];
    a.out = n->gbuf[1 - cur];
    a.mask = n->act[i];
    a.B = B;
    a.H = H;
    a.W = W;
    e = (i == 5) ? conv<8, 32, CONV_DGRAD>(a, st) : conv<32, 32, CONV_DGRAD>(a, st);
    cur = 1 - cur;
  }
  return e;
}

hipError_t pack_weights(ils_net* n) {
  PackArgs pa;
  pa.master = n->master;
  for (int i = 0; i < 6; ++i) {
    pa.wf[i] = n->wf[i];
    pa.wd[i] = n->wd[i];
    pa.bias[i] = n->bias[i];
  }
  hipLaunchKernelGGL(k_pack_weights, dim3(16, 6), dim3(256), 0, n->stream, pa);
  return hipGetLastError();
}

int check_batch(const ils_net* n, int B, int H, int W) {
  if (B < 1 || H < 2 || W < 2 || B > n->max_B || H > n->max_H || W > n->max_W) return ILS_ERR_INVALID_ARG;
  if (B > 512) return ILS_ERR_INVALID_ARG;
  return ILS_OK;
}

}  // namespace

// ------------------------------------------------------------------ C ABI
extern "C" {

int ils_net_param_count(void) { return (int)kNet.nparams; }

size_t ils_net_workspace_bytes(int max_B, int max_H, int max_W) {
  if (max_B < 1 || max_H < 2 || max_W < 2) return 0;
  return net_layout(max_B, max_H, max_W, nullptr);
}

int ils_net_create(ils_net** out, int max_B, int max_H, int max_W, void* workspace, size_t ws_bytes,
                   void* hip_stream) {
  if (!out) return ILS_ERR_INVALID_ARG;
  *out = nullptr;
  if (max_B < 1 || max_H < 2 || max_W < 2) return ILS_ERR_INVALID_ARG;
  if (!workspace || ((uintptr_t)workspace & 255)) return ILS_ERR_WORKSPACE;
  if (ws_bytes < ils_net_workspace_bytes(max_B, max_H, max_W)) return ILS_ERR_WORKSPACE;
  ils_net* n = new (std::nothrow) ils_net();
  if (!n) return ILS_ERR_HIP;
  n->max_B = max_B;
  n->max_H = max_H;
  n->max_W = max_W;
  n->stream = static_cast<hipStream_t>(hip_stream);
  n->ws = static_cast<char*>(workspace);
  n->ws_bytes = ws_bytes;
  n->last_error = ILS_OK;
  n->step = 0;
  net_layout(max_B, max_H, max_W, n);
  *out = n;
  return ILS_OK;
}

int ils_net_set_stream(ils_net* n, void* hip_stream) {
  if (!n) return ILS_ERR_INVALID_ARG;
  n->stream = static_cast<hipStream_t>(hip_stream);
  return ILS_OK;
}

int ils_net_set_state(ils_net* n, const float* params, const float* m, const float* v, long long step) {
  if (!n || !params || step < 0) return ILS_ERR_INVALID_ARG;
  const size_t bytes = kNet.nparams * 4;
  hipError_t e = hipMemcpy(n->master, params, bytes, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = m ? hipMemcpy(n->adam_m, m, bytes, hipMemcpyHostToDevice) : hipMemset(n->adam_m, 0, bytes);
  if (e == hipSuccess) e = v ? hipMemcpy(n->adam_v, v, bytes, hipMemcpyHostToDevice) : hipMemset(n->adam_v, 0, bytes);
  if (e == hipSuccess) e = pack_weights(n);
  if (e == hipSuccess) e = hipStreamSynchronize(n->stream);
  n->step = step;
  return rec(n, e);
}

int ils_net_get_state(ils_net* n, float* params, float* m, float* v, long long* step) {
  if (!n) return ILS_ERR_INVALID_ARG;
  const size_t bytes = kNet.nparams * 4;
  hipError_t e = hipStreamSynchronize(n->stream);
  if (e == hipSuccess && params) e = hipMemcpy(params, n->master, bytes, hipMemcpyDeviceToHost);
  if (e == hipSuccess && m) e = hipMemcpy(m, n->adam_m, bytes, hipMemcpyDeviceToHost);
  if (e == hipSuccess && v) e = hipMemcpy(v, n->adam_v, bytes, hipMemcpyDeviceToHost);
  if (step) *step = n->step;
  return rec(n, e);
}

int ils_net_forward(ils_net* n, const float* f, const float* lam, const float* p, int B, int H, int W, float* v) {
  if (!n || !f || !lam || !p || !v) return ILS_ERR_INVALID_ARG;
  int rc = check_batch(n, B, H, W);
  if (rc != ILS_OK) return rc;
  return rec(n, run_forward(n, f, lam, p, B, H, W, v));
}

int ils_net_gradients(ils_net* n, const float* f, const float* lam, const float* p, const float* target, int B, int H,
                      int W, float* grad, float* loss) {
  if (!n || !f || !lam || !p || !target || !grad || !loss) return ILS_ERR_INVALID_ARG;
  int rc = check_batch(n, B, H, W);
  if (rc != ILS_OK) return rc;
  hipError_t e = run_forward(n, f, lam, p, B, H, W, n->zbuf);
  if (e == hipSuccess) e = run_backward(n, target, B, H, W);
  if (e == hipSuccess) e = hipMemcpyAsync(grad, n->grad, kNet.nparams * 4, hipMemcpyDeviceToDevice, n->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(loss, n->loss, 4, hipMemcpyDeviceToDevice, n->stream);
  return rec(n, e);
}

int ils_net_train_step(ils_net* n, const float* f, const float* lam, const float* p, const float* target, int B,
                       int H, int W, float lr, float* loss) {
  if (!n || !f || !lam || !p || !target) return ILS_ERR_INVALID_ARG;
  if (!(lr > 0.0f) || !std::isfinite(lr)) return ILS_ERR_INVALID_ARG;
  int rc = check_batch(n, B, H, W);
  if (rc != ILS_OK) return rc;
  hipError_t e = run_forward(n, f, lam, p, B, H, W, n->zbuf);
  if (e == hipSuccess) e = run_backward(n, target, B, H, W);
  if (e == hipSuccess) {
    n->step += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = (float)(1.0 - std::pow(0.9, (double)n->step));
    const float c2 = (float)(1.0 - std::pow(0.999, (double)n->step));
    const int np = (int)kNet.nparams;
    hipLaunchKernelGGL(k_adam, dim3((np + 255) / 256), dim3(256), 0, n->stream, n->master, n->adam_m, n->adam_v,
                       n->grad, np, lr, b1, b2, 1e-8f, c1, c2);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = pack_weights(n);
  if (e == hipSuccess && loss) e = hipMemcpyAsync(loss, n->loss, 4, hipMemcpyDeviceToDevice, n->stream);
  return rec(n, e);
}

int ils_net_last_error(ils_net* n) {
  if (!n) return ILS_ERR_INVALID_ARG;
  int r = n->last_error;
  n->last_error = ILS_OK;
  return r;
}

int ils_net_destroy(ils_net* n) {
  delete n;
  return ILS_OK;
}

// Residual-gated surrogate inference.  v = net(f); for every image
// T(v) = one ILS iteration from u^0 = v with data term f; R = rms(T(v) - v);
// images with R > tau are recomputed with plain ILS (N iterations) into out.
// The gated pipeline proper; the plan is already bound to the network's stream.
static int surrogate_infer_bound(ils_net* n, ils_plan* plan, const float* f, const float* lam_dev, const float* p_dev,
                                 const float* lam_host, const float* p_host, float eps, int N, int B, int H, int W,
                                 float tau, float* out, float* tv_scratch, float* residual_host, int* fallback_host) {
  int rc = ILS_OK;
  hipError_t e = run_forward(n, f, lam_dev, p_dev, B, H, W, out);
  if (e != hipSuccess) return rec(n, e);
  const size_t img = (size_t)3 * H * W;
  std::vector<const float*> pa(B), pb(B);
  std::vector<long long> cnt(B, (long long)img);
  // T(v) for every image: one batched call when the plan holds B frames of
  // this size (every argument was checked above, so a refusal can only be
  // the plan's frame count or workspace), else image by image; both give
  // the same bits.
  std::vector<ils_frame> tv(B);
  for (int b = 0; b < B; ++b) {
    tv[b] = ils_frame{f + b * img, tv_scratch + b * img, H, W, 3, lam_host[b], p_host[b], eps, 1, out + b * img,
                      ILS_PENALTY_CHARBONNIER, 0.0f};
    pa[b] = tv_scratch + b * img;
    pb[b] = out + b * img;
  }
  rc = ils_smooth_batch(plan, tv.data(), B);
  if (rc == ILS_ERR_WORKSPACE || rc == ILS_ERR_INVALID_ARG) {
    for (int b = 0; b < B; ++b) {
      rc = ils_iterate_from(plan, f + b * img, out + b * img, H, W, 3, lam_host[b], p_host[b], eps, 1,
                            tv_scratch + b * img);
      if (rc != ILS_OK) return rc;
    }
  }
  if (rc != ILS_OK) return rc;
  // per-image residuals go to the loss-partial area of the network workspace
  float* rms_dev = reinterpret_cast<float*>(n->lpart);
  rc = ils_rms_diff(plan, pa.data(), pb.data(), cnt.data(), B, rms_dev);
  if (rc != ILS_OK) return rc;
  e = hipMemcpyAsync(residual_host, rms_dev, B * sizeof(float), hipMemcpyDeviceToHost, n->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(n->stream);
  if (e != hipSuccess) return rec(n, e);
  std::vector<ils_frame> fb;
  for (int b = 0; b < B; ++b) {
    fallback_host[b] = !(residual_host[b] <= tau);  // NaN residual also falls back
    if (fallback_host[b])
      fb.push_back(ils_frame{f + b * img, out + b * img, H, W, 3, lam_host[b], p_host[b], eps, N, nullptr,
                             ILS_PENALTY_CHARBONNIER, 0.0f});
  }
  if (fb.empty()) return ILS_OK;
  // plain ILS for the images that fall back, batched like T(v) when the plan allows
  rc = ils_smooth_batch(plan, fb.data(), (int)fb.size());
  if (rc == ILS_ERR_WORKSPACE || rc == ILS_ERR_INVALID_ARG) {
    for (const ils_frame& fr : fb) {
      rc = ils_smooth(plan, fr.f, H, W, 3, fr.lambda, fr.p, eps, N, fr.out);
      if (rc != ILS_OK) return rc;
    }
    rc = ILS_OK;
  }
  return rc;
}

// Frame-list gate: the network frame by frame (its lambda and p maps from two
// scalars that a one-thread kernel writes into the workspace, so the host
// stages nothing), then T(v), the residuals and the fallback over the whole
// list, as in surrogate_infer_bound.
static int surrogate_infer_frames_bound(ils_net* n, ils_plan* plan, const ils_frame* frames, int nf, float tau,
                                        float* tv_scratch, float* residual_host, int* fallback_host) {
  float* lp = reinterpret_cast<float*>(n->lpart);  // lambda, p of the frame in flight
  std::vector<ils_frame> tv(nf);
  std::vector<const float*> pa(nf), pb(nf);
  std::vector<long long> cnt(nf);
  size_t off = 0;
  for (int i = 0; i < nf; ++i) {
    const ils_frame& fr = frames[i];
    hipLaunchKernelGGL(k_set_pair, dim3(1), dim3(64), 0, n->stream, lp, fr.lambda, fr.p);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = run_forward(n, fr.f, lp, lp + 1, 1, fr.H, fr.W, fr.out);
    if (e != hipSuccess) return rec(n, e);
    const size_t img = (size_t)3 * fr.H * fr.W;
    tv[i] = ils_frame{fr.f, tv_scratch + off, fr.H, fr.W, 3, fr.lambda, fr.p, fr.eps, 1, fr.out,
                      ILS_PENALTY_CHARBONNIER, 0.0f};
    pa[i] = tv_scratch + off;
    pb[i] = fr.out;
    cnt[i] = (long long)img;
    off += img;
  }
  int rc = ils_smooth_batch(plan, tv.data(), nf);
  if (rc == ILS_ERR_WORKSPACE || rc == ILS_ERR_INVALID_ARG) {
    for (const ils_frame& t : tv) {
      rc = ils_iterate_from(plan, t.f, t.u0, t.H, t.W, 3, t.lambda, t.p, t.eps, 1, t.out);
      if (rc != ILS_OK) return rc;
    }
  }
  if (rc != ILS_OK) return rc;
  float* rms_dev = reinterpret_cast<float*>(n->lpart);
  rc = ils_rms_diff(plan, pa.data(), pb.data(), cnt.data(), nf, rms_dev);
  if (rc != ILS_OK) return rc;
  hipError_t e = hipMemcpyAsync(residual_host, rms_dev, nf * sizeof(float), hipMemcpyDeviceToHost, n->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(n->stream);
  if (e != hipSuccess) return rec(n, e);
  std::vector<ils_frame> fb;
  for (int i = 0; i < nf; ++i) {
    fallback_host[i] = !(residual_host[i] <= tau);  // NaN residual also falls back
    if (fallback_host[i]) {
      const ils_frame& fr = frames[i];
      fb.push_back(ils_frame{fr.f, fr.out, fr.H, fr.W, 3, fr.lambda, fr.p, fr.eps, fr.N, nullptr,
                             ILS_PENALTY_CHARBONNIER, 0.0f});
    }
  }
  if (fb.empty()) return ILS_OK;
  rc = ils_smooth_batch(plan, fb.data(), (int)fb.size());
  if (rc == ILS_ERR_WORKSPACE || rc == ILS_ERR_INVALID_ARG) {
    for (const ils_frame& fr : fb) {
      rc = ils_smooth(plan, fr.f, fr.H, fr.W, 3, fr.lambda, fr.p, fr.eps, fr.N, fr.out);
      if (rc != ILS_OK) return rc;
    }
    rc = ILS_OK;
  }
  return rc;
}

int ils_surrogate_infer_frames(ils_net* n, ils_plan* plan, const ils_frame* frames, int nframes, float tau,
                               float* tv_scratch, float* residual_host, int* fallback_host) {
  if (!n || !plan || !frames || !tv_scratch || !residual_host || !fallback_host) return ILS_ERR_INVALID_ARG;
  if (nframes < 1 || nframes > n->max_B) return ILS_ERR_INVALID_ARG;
  if (!std::isfinite(tau)) return ILS_ERR_NOT_CALIBRATED;
  for (int i = 0; i < nframes; ++i) {
    const ils_frame& fr = frames[i];
    if (!fr.f || !fr.out || fr.C != 3 || fr.penalty != ILS_PENALTY_CHARBONNIER || (fr.u0 && fr.u0 != fr.f))
      return ILS_ERR_INVALID_ARG;
    int rc = check_batch(n, 1, fr.H, fr.W);
    if (rc == ILS_OK) rc = ils_check_args(fr.H, fr.W, 3, fr.lambda, fr.p, fr.eps, fr.N);
    if (rc != ILS_OK) return rc;
  }
  void* saved = ilsk_plan_stream(plan);
  int rc = ils_plan_set_stream(plan, n->stream);
  if (rc != ILS_OK) return rc;
  rc = surrogate_infer_frames_bound(n, plan, frames, nframes, tau, tv_scratch, residual_host, fallback_host);
  (void)ils_plan_set_stream(plan, saved);
  return rc;
}

int ils_surrogate_infer(ils_net* n, ils_plan* plan, const float* f, const float* lam_dev, const float* p_dev,
                        const float* lam_host, const float* p_host, float eps, int N, int B, int H, int W,
                        float tau, float* out, float* tv_scratch, float* residual_host, int* fallback_host) {
  if (!n || !plan || !f || !lam_dev || !p_dev || !lam_host || !p_host || !out || !tv_scratch || !residual_host ||
      !fallback_host)
    return ILS_ERR_INVALID_ARG;
  if (!std::isfinite(tau)) return ILS_ERR_NOT_CALIBRATED;
  int rc = check_batch(n, B, H, W);
  if (rc != ILS_OK) return rc;
  for (int b = 0; b < B; ++b) {
    rc = ils_check_args(H, W, 3, lam_host[b], p_host[b], eps, N);
    if (rc != ILS_OK) return rc;
  }
  // the plan's own work goes on the network's stream for the call and back
  // to the caller's stream on every return path
  void* saved = ilsk_plan_stream(plan);
  rc = ils_plan_set_stream(plan, n->stream);
  if (rc != ILS_OK) return rc;
  rc = surrogate_infer_bound(n, plan, f, lam_dev, p_dev, lam_host, p_host, eps, N, B, H, W, tau, out, tv_scratch,
                             residual_host, fallback_host);
  (void)ils_plan_set_stream(plan, saved);
  return rc;
}

}  // extern "C"
