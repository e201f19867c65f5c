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
#include <utility>

namespace ilsn {

typedef __bf16 bf16;
typedef bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

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

__device__ __forceinline__ int imin(int a, int b) { return a < b ? a : b; }

// v mod n for -n <= v < 2n.
__device__ __forceinline__ int wrap1(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

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

constexpr int kXcds = 8;  // workgroup b of a launch runs on accelerator die b mod 8

// Tiles: an image is cut into tiles_y x tiles_x output tiles of th x tw
// pixels; tile t of the batch is image t / (tiles_y tiles_x), row-major
// within it.  The grid is sized to what the chip holds at once, so that a
// workgroup loads the weight fragments into registers once and fetches the
// next tile's halo into registers while it computes on the current one.
// Each die takes one contiguous run of tiles (whole stripes of tile rows),
// walked by its workgroups in step, so that the halo a tile shares with its
// neighbours above, below and beside it is read once into that die's L2.
struct TileGrid {
  int tiles_x, per_img, ntiles, th, tw;
  __device__ TileGrid(int B, int H, int W, int th_, int tw_) : th(th_), tw(tw_) {
    tiles_x = (W + tw - 1) / tw;
    per_img = tiles_x * ((H + th - 1) / th);
    ntiles = B * per_img;
  }
  // tiles t0, t0 + step, ... below t_end of this workgroup
  __device__ void span(int& t0, int& t_end, int& step) const {
    const int G = gridDim.x, b = blockIdx.x;
    if (G % kXcds == 0) {
      const int x = b % kXcds, per = (ntiles + kXcds - 1) / kXcds;
      t0 = x * per + b / kXcds;
      t_end = per * (x + 1) < ntiles ? per * (x + 1) : ntiles;
      step = G / kXcds;
    } else {
      t0 = b;
      t_end = ntiles;
      step = G;
    }
  }
  __device__ void origin(int t, int& img, int& y0, int& x0) const {
    img = t / per_img;
    const int r = t - img * per_img;
    const int ty = r / tiles_x;
    y0 = ty * th;
    x0 = (r - ty * tiles_x) * tw;
  }
};

// LH x LW pixels of CIP channels around (y0 - HALO, x0 - HALO), periodic,
// held in registers as 16-byte chunks; chunk i goes to LDS element 8 i.
// Chunk j of a thread is chunk threadIdx.x + j NTHREADS of the tile; every
// access to r[] has a compile-time index so that r[] stays in registers.
template <int CIP, int LH, int LW, int HALO>
struct TileStage {
  static constexpr int CH16 = CIP / 8;
  static constexpr int TOTAL = LH * LW * CH16;
  static constexpr int NLD = (TOTAL + NTHREADS - 1) / NTHREADS;
  u32x4 r[NLD];

  // Every lane issues every load (past the end of the tile it loads the
  // tile's last chunk again and does not store it), so that the loads form
  // one branch-free sequence.  NEAR: the image is at least LH x LW, so a
  // halo coordinate is off by at most one period.
  template <int J, bool NEAR>
  __device__ __forceinline__ void fetch_one(const bf16* in, int H, int W, int y0, int x0) {
    const int i = imin(threadIdx.x + J * NTHREADS, TOTAL - 1);
    const int pix = i / CH16, chn = i - pix * CH16;
    const int ly = pix / LW, lx = pix - ly * LW;
    const int gy = NEAR ? wrap1(y0 + ly - HALO, H) : wrapi(y0 + ly - HALO, H);
    const int gx = NEAR ? wrap1(x0 + lx - HALO, W) : wrapi(x0 + lx - HALO, W);
    r[J] = *reinterpret_cast<const u32x4*>(&in[((size_t)gy * W + gx) * CIP + chn * 8]);
  }
  template <int J>
  __device__ __forceinline__ void store_one(bf16* tile) const {
    const int i = threadIdx.x + J * NTHREADS;
    if (J * NTHREADS + NTHREADS <= TOTAL || i < TOTAL) *reinterpret_cast<u32x4*>(&tile[i * 8]) = r[J];
  }
  template <bool NEAR, int... J>
  __device__ __forceinline__ void fetch_all(std::integer_sequence<int, J...>, const bf16* in, int H, int W, int y0,
                                            int x0) {
    (fetch_one<J, NEAR>(in, H, W, y0, x0), ...);
  }
  template <int... J>
  __device__ __forceinline__ void store_all(std::integer_sequence<int, J...>, bf16* tile) const {
    (store_one<J>(tile), ...);
  }

  // tile t of the grid, from the batch tensor `in` (B images of H x W)
  template <bool NEAR>
  __device__ __forceinline__ void fetch_tile(const TileGrid& tg, const bf16* in, int H, int W, int t) {
    int img, y0, x0;
    tg.origin(t, img, y0, x0);
    fetch_all<NEAR>(std::make_integer_sequence<int, NLD>{}, in + (size_t)img * H * W * CIP, H, W, y0, x0);
  }
  __device__ __forceinline__ void store(bf16* tile) const { store_all(std::make_integer_sequence<int, NLD>{}, tile); }
};

template <int CIP, int COP>
__device__ __forceinline__ void load_wfrag(const bf16* wfrag, bf16x8 (&wf)[COP / 16][kpad(CIP) / 32]) {
  constexpr int KP = kpad(CIP);
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int mb = 0; mb < COP / 16; ++mb)
#pragma unroll
    for (int kb = 0; kb < KP / 32; ++kb)
      wf[mb][kb] = *reinterpret_cast<const bf16x8*>(&wfrag[(mb * 16 + (lane & 15)) * KP + kb * 32 + (lane >> 4) * 8]);
}

// acc[r][nb][mb] = W x X for the output pixels (row0 + r, 16 nb + lane % 16)
// of a tile in LDS whose rows are LW pixels of CIP channels; the tap (a, c)
// of output (y, x) reads tile pixel (y + a, x + c).
template <int CIP, int COP, int LW>
__device__ __forceinline__ void conv_mfma(const bf16* tile, const bf16x8 (&wf)[COP / 16][kpad(CIP) / 32], int row0,
                                          f32x4 (&acc)[2][2][COP / 16]) {
  constexpr int KB = kpad(CIP) / 32;
  constexpr int MB = COP / 16;
  const int lane = threadIdx.x & 63;
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
        const int ly = row0 + r + ta;
        const int lx = nb * 16 + (lane & 15) + tc;
        const bf16x8 bfr = *reinterpret_cast<const bf16x8*>(&tile[(ly * LW + lx) * CIP + chunk * 8]);
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
          acc[r][nb][mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wf[mb][kb], bfr, acc[r][nb][mb], 0, 0, 0);
      }
    }
  }
}

// NEAR: the image is at least (TH + 2) x (TW + 2) (chosen by the launcher).
template <int CIP, int COP, int MODE, bool NEAR>
__global__ void __launch_bounds__(NTHREADS) __attribute__((amdgpu_waves_per_eu(MODE == CONV_LAST ? 3 : 1))) k_conv(ConvArgs a) {
  constexpr int LH = TH + 2, LW = TW + 2;
  constexpr int MB = COP / 16;
  constexpr int TILE = LH * LW * CIP;
  // tiles whose halo is in flight in registers (the last layer keeps one so
  // that three wavefronts per SIMD still fit)
  constexpr int DEPTH = (MODE == CONV_LAST) ? 1 : 2;
  __shared__ __attribute__((aligned(16))) bf16 tile[2 * TILE];  // double-buffered halo tile

  const int H = a.H, W = a.W;
  const TileGrid tg(a.B, H, W, TH, TW);
  const size_t plane = (size_t)H * W;
  int t, t_end, G;
  tg.span(t, t_end, G);
  if (t >= t_end) return;
  const int last = t_end - 1;
  using Stage = TileStage<CIP, LH, LW, 1>;
  Stage st[DEPTH];
  st[0].template fetch_tile<NEAR>(tg, a.in, H, W, t);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  bf16x8 wf[MB][kpad(CIP) / 32];
  load_wfrag<CIP, COP>(a.wfrag, wf);
  float bias[MB][4];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int i = 0; i < 4; ++i) bias[mb][i] = (MODE == CONV_DGRAD) ? 0.0f : a.bias[mb * 16 + 4 * (lane >> 4) + i];
  st[0].store(tile);
  __syncthreads();
  // Every prefetch is issued (past the end it repeats the last tile), so
  // the number of loads in flight behind a stage is the same on every path
  // and waiting for one stage never waits for the next one's loads.
#pragma unroll
  for (int k = 0; k < DEPTH; ++k) st[k].template fetch_tile<NEAR>(tg, a.in, H, W, imin(t + (k + 1) * G, last));

  // One tile: t is in LDS buffer cur, nx holds tile t + G.  The next tile's
  // halo is stored to the other LDS buffer before this tile's results go
  // out, so that waiting for its loads never waits for this tile's stores
  // (one counter covers both); nx then fetches tile t + (DEPTH + 1) G.
  auto step = [&](Stage& nx, int cur) __attribute__((always_inline)) -> bool {
    int img, y0, x0;
    tg.origin(t, img, y0, x0);
    // CONV_LAST: this tile's f, loaded before the MFMAs so that it arrives during them
    float fpix[2][2][3];
    if constexpr (MODE == CONV_LAST) {
#pragma unroll
      for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) {
          const int y = y0 + wave * 2 + r, x = x0 + nb * 16 + (lane & 15);
          const bool in = (lane >> 4) == 0 && y < H && x < W;
          const size_t base = (size_t)img * 3 * plane + (size_t)(in ? y : 0) * W + (in ? x : 0);
#pragma unroll
          for (int i = 0; i < 3; ++i) fpix[r][nb][i] = in ? a.f[base + i * plane] : 0.0f;
        }
    }
    f32x4 acc[2][2][MB];
    conv_mfma<CIP, COP, LW>(tile + cur * TILE, wf, wave * 2, acc);
    if (t + G < t_end) nx.store(tile + (cur ^ 1) * TILE);

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
            for (int i = 0; i < 4; ++i) o[i] = f2bf(fmaxf(d[i] + bias[mb][i], 0.0f));
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
              for (int i = 0; i < 3; ++i) a.v[base + i * plane] = fpix[r][nb][i] + d[i] + bias[0][i];
            }
          }
        }
      }
    }
    __syncthreads();  // the other buffer is complete; every wave is done with this one
    nx.template fetch_tile<NEAR>(tg, a.in, H, W, imin(t + (DEPTH + 1) * G, last));
    t += G;
    return t < t_end;
  };
  if constexpr (DEPTH == 1) {
    for (int cur = 0; step(st[0], cur); cur ^= 1) {
    }
  } else {
    while (step(st[0], 0) && step(st[DEPTH - 1], 1)) {
    }
  }
}

}  // namespace ilsn
