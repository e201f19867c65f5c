// Per-frame descriptor shared by the host planner and the kernels.
#pragma once

#include <cstdint>

// Global (address space 1) qualifier for device pointers.  Pointers that
// reach a kernel inside a descriptor are otherwise generic, and the compiler
// then emits FLAT memory instructions, which also count against the LDS
// wait counter: every wait for an LDS result would wait for outstanding
// image and spectrum loads too.
// (The host pass of the compiler parses the device code too; there the
// qualifier means nothing and is left out.)
#if defined(__HIP_DEVICE_COMPILE__)
#define ILS_G __attribute__((address_space(1)))
#else
#define ILS_G
#endif

namespace ilsk {

template <class T>
__host__ __device__ __forceinline__ ILS_G T* gm(T* p) {
  return (ILS_G T*)p;
}

struct cf;

// One frame (all of its channels) of one ILS call.  Layouts:
//   f, u0, out : C x H x W float32, row-major, channel stride H*W
//   specA/specB: C x H x ldS complex64 (half spectrum, W/2+1 used columns
//                per row, ldS >= W/2+1), channel stride H*ldS
// The row passes read specB and write specA; the column pass reads specA
// and writes specB.
struct FrameDesc {
  const float* f;    // data term of the LS problem
  const float* u0;   // first iterate (normally == f)
  float* out;        // result u^N
  cf* specA;
  cf* specB;
  const cf* tw_row;   // exp(-2 pi i j / M), j < M          (M = W/2)
  const cf* tw2_row;  // exp(-pi i k / M),  k <= M
  const cf* twm_row;  // exp(-2 pi i t k1 / M) at [k1 * (Q|1) + t], M = P Q
  const float* sx;    // 4 sin^2(pi k / W), k <= M
  const cf* tw_col;   // exp(-2 pi i j / H), j < H
  const cf* twm_col;  // exp(-2 pi i j k1 / H) at [k1 * (Q|1) + j], H = P Q
  const float* sy;    // 4 sin^2(pi l / H), l < H
  int H, W, C, ldS;
  float kappa;      // lambda * c / 2, c >= c0 = p eps^(p/2 - 1) (Welsch: c = 2)
  float a_exp;      // p/2 - 1 (Welsch: -log2(e) / (2 gamma^2))
  float inv_eps;    // 1 / eps (Welsch: unused)
  float log2_r;     // log2(c0 / c): 0 for the paper's c = c0
  float col_scale;  // 1 / (2 H W): inverse-transform normalisation (and the
                    // factor 2 the row R2C leaves in its output)
  float boost;      // final pass writes u + boost (f - u) when non-zero
                    // (detail enhancement); 0 writes u
  int nb_row;       // row bands per channel (0: as many as bands of the
                    // kernel's full height need); see row_bands
};

// Bands of the row passes.  A channel's H rows are split into nb bands, band
// b holding rows [b H / nb, (b + 1) H / nb) (floor or ceil of H / nb rows);
// nb is the frame's own count, kept within [ceil(H / G), H] so that no band
// exceeds the G rows a block holds.
__host__ __device__ inline int row_bands(const FrameDesc& d, int G) {
  const int lo = (d.H + G - 1) / G;
  const int nb = d.nb_row > lo ? d.nb_row : lo;
  return nb < d.H ? nb : d.H;
}

// ROW_FIRST_SAME is the first pass when u^0 and f are the same image (the
// data term is then read once, as u^0).
enum RowMode : int { ROW_FIRST = 0, ROW_MID = 1, ROW_FINAL = 2, ROW_FIRST_SAME = 3 };

}  // namespace ilsk
