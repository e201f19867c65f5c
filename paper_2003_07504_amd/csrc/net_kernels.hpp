// Kernels of the learned surrogate: six periodic 3x3 convolutions, 32
// channels, ReLU after the first five, output v = f + z6.  Weights and
// activations are bf16, accumulation is fp32 on the MFMA units
// (v_mfma_f32_16x16x32_bf16), master weights and optimiser state fp32.
//
// Tensors:
//   x0        NHWC bf16, 8 channels: (r, g, b, lambda, p, 0, 0, 0)
//   a1 .. a5  NHWC bf16, 32 channels (post-ReLU)
//   g         NHWC bf16 gradients with the channel count of the forward
//             output they belong to (32, or 8 for the 3-channel output)
//   f, v, t   planar fp32 (B, 3, H, W)
// Weight fragments (bf16) for a convolution with CIP input and COP output
// channels: WF[co][k], k = tap * CIP + ci, tap = 3 a + c, padded to KP =
// ceil(9 CIP / 32) * 32 columns and COP rows (zeros outside the layer).
//
// A convolution is an implicit GEMM D[co][pixel] = sum_k WF[co][k] X[k][pixel]
// with X[tap*CIP + ci][(y, x)] = in[(y + a - 1) mod H][(x + c - 1) mod W][ci].
// MFMA 16x16x32 lane layout used: lane l supplies A[l % 16][8 (l/16) .. +8],
// B[8 (l/16) .. +8][l % 16] and receives D[4 (l/16) + i][l % 16], i < 4.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ilsn {

typedef __bf16 bf16;
typedef bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int TH = 8;   // output rows per convolution block (2 per wave)
constexpr int TW = 32;  // output columns per block (2 blocks of 16 pixels)
constexpr int NTHREADS = 256;

enum ConvMode : int { CONV_RELU = 0, CONV_LAST = 1, CONV_DGRAD = 2 };

__host__ __device__ constexpr int kpad(int cip) { return (9 * cip + 31) / 32 * 32; }

__device__ __forceinline__ float bf2f(bf16 v) { return (float)v; }

// Round to nearest even.
__device__ __forceinline__ bf16 f2bf(float v) { return (bf16)v; }

// v mod n in [0, n) for any v (halo tiles may be wider than the image).
__device__ __forceinline__ int wrapi(int v, int n) {
  int r = v % n;
  return r < 0 ? r + n : r;
}

struct ConvArgs {
  const bf16* in;       // NHWC, CIP channels
  const bf16* wfrag;    // COP x KP
  const float* bias;    // COP (zeros past the layer's channels); unused for DGRAD
  bf16* out;            // NHWC, COP channels (RELU, DGRAD)
  const bf16* mask;     // DGRAD: forward activation at this position (NHWC, COP channels)
  const float* f;       // LAST: planar fp32 input image (B, 3, H, W)
  float* v;             // LAST: planar fp32 output (B, 3, H, W)
  int B, H, W;
};

template <int CIP, int COP, int MODE>
__global__ void __launch_bounds__(NTHREADS) k_conv(ConvArgs a) {
  constexpr int LH = TH + 2, LW = TW + 2;
  constexpr int KP = kpad(CIP);
  constexpr int KB = KP / 32;
  constexpr int MB = COP / 16;
  constexpr int CH16 = CIP / 8;  // 16-byte chunks per pixel
  __shared__ __attribute__((aligned(16))) bf16 tile[LH * LW * CIP];

  const int H = a.H, W = a.W;
  const int tiles_x = (W + TW - 1) / TW, tiles_y = (H + TH - 1) / TH;
  int bid = blockIdx.x;
  const int img = bid / (tiles_x * tiles_y);
  bid -= img * tiles_x * tiles_y;
  const int ty = bid / tiles_x, tx = bid - ty * tiles_x;
  const int y0 = ty * TH, x0 = tx * TW;
  const size_t plane = (size_t)H * W;
  const bf16* in = a.in + (size_t)img * plane * CIP;

  // halo tile, periodic in both directions
  for (int i = threadIdx.x; i < LH * LW * CH16; i += NTHREADS) {
    const int pix = i / CH16, chn = i - pix * CH16;
    const int ly = pix / LW, lx = pix - ly * LW;
    const int gy = wrapi(y0 + ly - 1, H), gx = wrapi(x0 + lx - 1, W);
    *reinterpret_cast<uint4*>(&tile[pix * CIP + chn * 8]) =
        *reinterpret_cast<const uint4*>(&in[((size_t)gy * W + gx) * CIP + chn * 8]);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  bf16x8 wf[MB][KB];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int kb = 0; kb < KB; ++kb)
      wf[mb][kb] = *reinterpret_cast<const bf16x8*>(&a.wfrag[(mb * 16 + (lane & 15)) * KP + kb * 32 + (lane >> 4) * 8]);
  __syncthreads();

  f32x4 acc[2][2][MB];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int nb = 0; nb < 2; ++nb)
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) acc[r][nb][mb] = f32x4{0.f, 0.f, 0.f, 0.f};

#pragma unroll
  for (int kb = 0; kb < KB; ++kb) {
    int tap, chunk;
    if constexpr (CIP == 32) {
      tap = kb;
      chunk = lane >> 4;
    } else {  // CIP == 8: one K block = four taps of 8 channels
      tap = kb * 4 + (lane >> 4);
      if (tap > 8) tap = 8;  // zero weights there; any finite operand will do
      chunk = 0;
    }
    const int ta = tap / 3, tc = tap - 3 * ta;
#pragma unroll
    for (int r = 0; r < 2; ++r) {
#pragma unroll
      for (int nb = 0; nb < 2; ++nb) {
        const int ly = wave * 2 + r + ta;
        const int lx = nb * 16 + (lane & 15) + tc;
        const bf16x8 bfr = *reinterpret_cast<const bf16x8*>(&tile[(ly * LW + lx) * CIP + chunk * 8]);
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
          acc[r][nb][mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wf[mb][kb], bfr, acc[r][nb][mb], 0, 0, 0);
      }
    }
  }

  // epilogue: lane holds co = mb*16 + 4*(lane/16) + i of pixel (row r, column nb*16 + lane%16)
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const int y = y0 + wave * 2 + r;
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) {
      const int x = x0 + nb * 16 + (lane & 15);
      if (y >= H || x >= W) continue;
      const size_t pix = (size_t)img * plane + (size_t)y * W + x;
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) {
        const int co0 = mb * 16 + 4 * (lane >> 4);
        const f32x4 d = acc[r][nb][mb];
        if constexpr (MODE == CONV_RELU) {
          bf16 o[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) o[i] = f2bf(fmaxf(d[i] + a.bias[co0 + i], 0.0f));
          *reinterpret_cast<uint2*>(&a.out[pix * COP + co0]) = *reinterpret_cast<const uint2*>(o);
        } else if constexpr (MODE == CONV_DGRAD) {
          const uint2 mraw = *reinterpret_cast<const uint2*>(&a.mask[pix * COP + co0]);
          const bf16* m = reinterpret_cast<const bf16*>(&mraw);
          bf16 o[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) o[i] = f2bf(bf2f(m[i]) > 0.0f ? d[i] : 0.0f);
          *reinterpret_cast<uint2*>(&a.out[pix * COP + co0]) = *reinterpret_cast<const uint2*>(o);
        } else {  // CONV_LAST: v = f + z for the three image channels
          if (co0 == 0) {
            const size_t base = (size_t)img * 3 * plane + (size_t)y * W + x;
#pragma unroll
            for (int i = 0; i < 3; ++i) a.v[base + i * plane] = a.f[base + i * plane] + d[i] + a.bias[i];
          }
        }
      }
    }
  }
}

}  // namespace ilsn
