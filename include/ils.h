/*
 * ils.h -- C ABI of the MI355X (gfx950) library for Iterative Least Squares
 * edge-preserving smoothing (Liu, Zhang, Huang, Yang, Shen, Reid: "Real-time
 * Image Smoothing via Iterative Least Squares").
 *
 * The library runs Algorithm 1 of the paper: starting from u^0 = f it
 * repeats N times
 *     mu^n = c nabla u^n - phi_p'(nabla u^n)                       Eq. (7)
 *     u^{n+1} = argmin_u sum (u - f)^2
 *               + lambda/2 sum (sqrt(c) nabla u - mu^n / sqrt(c))^2  Eq. (8)
 * with phi_p(x) = (x^2 + eps)^(p/2) (Eq. (2)), c = c0 = p eps^(p/2 - 1)
 * (Eq. (11), Sec. 3.3.3), nabla = periodic forward differences along x and
 * y (the [1, -1] kernels of Sec. 3), and the LS problem solved in the
 * Fourier domain under periodic boundaries (Eq. (9), Sec. 3.2) with one
 * real 2-D FFT and one inverse per iteration.  Colour images are smoothed
 * channel by channel (Sec. 3.4).  Arithmetic is float32.
 *
 * Conventions for every entry point:
 *   - Images are planar float32, C x H x W, row-major, contiguous, channel
 *     stride H*W.  Image pointers are DEVICE pointers owned by the caller.
 *   - Work is enqueued on the plan's HIP stream and the call returns after
 *     enqueue (asynchronous).  The caller synchronises the stream.
 *   - Every argument is validated before anything is enqueued; a non-zero
 *     status means nothing was enqueued.  Asynchronous HIP failures are
 *     reported by ils_last_error() after the stream has been synchronised.
 *   - The library never prints, throws or aborts.
 *   - A plan is not thread-safe: use one plan per host thread / stream.
 *   - Supported sizes: W even, and H and W/2 each a 2/3/5-smooth length
 *     from 2 to 4096, or one of the lengths compiled with a fixed four-step
 *     split (ils_length_supported).  A frame whose two lengths both have a
 *     compiled split runs the fused passes; any other supported frame runs
 *     runtime-length passes (mixed-radix Stockham transforms in LDS, the
 *     stencil step and the row transforms in separate kernels: 28 instead
 *     of 20 bytes per pixel-channel per iteration).  Other sizes return
 *     ILS_ERR_UNSUPPORTED_SIZE.
 */
#ifndef ILS_H_
#define ILS_H_

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define ILS_OK 0
#define ILS_ERR_INVALID_ARG -1      /* null pointer, bad range, NaN parameter   */
#define ILS_ERR_UNSUPPORTED_SIZE -2 /* H or W/2 not a supported length, W odd   */
#define ILS_ERR_WORKSPACE -3        /* workspace missing or too small           */
#define ILS_ERR_HIP -4              /* a HIP call failed (see ils_last_error)    */
#define ILS_ERR_NOT_CALIBRATED -5   /* surrogate gate used without a threshold  */

/* ils_plan_create flags. */
#define ILS_PLAN_NO_GRAPH 1u /* enqueue batched calls kernel by kernel (no graph) */

typedef struct ils_plan ils_plan;

/* Penalty functions of the smoothness term. */
#define ILS_PENALTY_CHARBONNIER 0 /* generalised Charbonnier phi_p, Eq. (2)    */
#define ILS_PENALTY_WELSCH 1      /* Welsch phi_W, Eq. (18), c = 2 (Eq. (20))  */

/* One frame of a batched call.  f / out: device pointers, C x H x W float32.
 * u0: device pointer of the first iterate, or NULL for u^0 = f (Alg. 1).
 * penalty: ILS_PENALTY_CHARBONNIER (uses p and eps; gamma ignored) or
 * ILS_PENALTY_WELSCH (uses gamma > 0; p and eps ignored).  A zeroed tail
 * (penalty = 0) selects the Charbonnier penalty. */
typedef struct ils_frame {
  const float* f;
  float* out;
  int H, W, C;
  float lambda, p, eps;
  int N;
  const float* u0;
  int penalty;
  float gamma;
} ils_frame;

/* Human-readable name of a status code (static string). */
const char* ils_status_string(int status);

/* 1 if L is a supported transform length (usable as H or as W/2): a
 * compiled length, or any 2/3/5-smooth L with 2 <= L <= 4096; else 0. */
int ils_length_supported(int L);

/* 1 if an H x W image is supported (W even, H and W/2 supported), else 0. */
int ils_size_supported(int H, int W);

/* Validation of ils_smooth's size and parameter arguments without a plan
 * (no HIP call): ILS_OK, ILS_ERR_INVALID_ARG or ILS_ERR_UNSUPPORTED_SIZE. */
int ils_check_args(int H, int W, int C, float lambda, float p, float eps, int N);

/* Bytes of device workspace a plan needs to smooth frames up to
 * max_H x max_W x max_C, max_frames of them resident at once (single-frame
 * calls use one slot).  Two half spectra (C x H x (W/2+1) complex64) per
 * frame plus alignment.  Returns 0 for invalid arguments. */
size_t ils_workspace_bytes(int max_H, int max_W, int max_C, int max_frames);

/* Exact workspace bytes ils_smooth_batch needs for this list of frames. */
size_t ils_batch_workspace_bytes(const ils_frame* frames, int n);

/* Create a plan.
 *   workspace / ws_bytes : caller-owned device memory (e.g. a torch uint8
 *                          tensor), 256-byte aligned, at least
 *                          ils_workspace_bytes(max_H, max_W, max_C, 1) bytes
 *                          (batched calls need ils_batch_workspace_bytes of
 *                          their frame list); it must outlive the plan.
 *   hip_stream           : hipStream_t to enqueue on (NULL = default stream).
 *   flags                : 0, or ILS_PLAN_NO_GRAPH.  By default the pass
 *                          sequence of a batched call is captured once as a
 *                          HIP graph and replayed while the batch structure
 *                          (sizes, channel counts, N) repeats.
 * The plan allocates only its own small device tables (FP64-computed
 * twiddles and Laplacian eigenvalues) and frees them in ils_plan_destroy.
 * Returns ILS_OK and sets *plan, or an error with *plan = NULL. */
int ils_plan_create(ils_plan** plan, int max_H, int max_W, int max_C, int max_frames,
                    void* workspace, size_t ws_bytes, void* hip_stream, unsigned flags);

/* Persistent single-launch sequences (SWITCHED OFF in this library).  The
 * design: for the sizes compiled with one (256 x 256, 640 x 480,
 * 1280 x 720, 1920 x 1080, 3840 x 2160), ils_smooth and the batched calls
 * would run the 2N + 1 passes of a frame (or of a part of a batch) in one
 * launch of a persistent grid: work items (row bands and column tiles, pass
 * by pass) taken from one queue, an item of a channel's pass waiting until
 * that channel's previous pass has completed, with results bitwise those of
 * the per-pass launches.  Its first launches on the MI355X did not end
 * (twice: once with waits bounded by a poll count, once with waits bounded
 * by the real-time clock), for a reason not found yet, so the path is off:
 * on = 0 is accepted (one launch per pass, the only mode), on = 1 returns
 * ILS_ERR_INVALID_ARG. */
int ils_plan_set_persistent(ils_plan* plan, int on);

/* Time a wait of a persistent launch may take before it gives up, in
 * microseconds (> 0), or the default (0: 20 ms).  For tests of the give-up
 * path: a limit of 1 us makes later items run before the items they depend
 * on have finished; the kernel still ends and ils_last_error then reports
 * ILS_ERR_HIP. */
int ils_plan_set_wait_limit(ils_plan* plan, long long microseconds);

/* Change the stream later work is enqueued on. */
int ils_plan_set_stream(ils_plan* plan, void* hip_stream);

/* Smooth one C x H x W frame: out = u^N of Algorithm 1 with u^0 = f.
 *   lambda >= 0 finite, 0 < p <= 2, eps > 0 finite, N >= 0.
 *   N == 0 or lambda == 0 copies f to out (u = f exactly).
 *   out == f (in place) is allowed; partial overlap is undefined.
 *   NaN/Inf in f propagate; the output is not clipped. */
int ils_smooth(ils_plan* plan, const float* f, int H, int W, int C, float lambda, float p,
               float eps, int N, float* out);

/* Smooth one frame with the Welsch penalty (Sec. 5): Algorithm 1 with the
 * pointwise step of Eq. (19), mu = c g - 2 g exp(-g^2 / (2 gamma^2)), and
 * c = c0 = 2 (Eq. (20)); the linear solve of Eq. (9) is unchanged.
 *   lambda >= 0 finite, gamma > 0 finite, N >= 0; other rules as ils_smooth.
 * The paper's settings: N = 10 for clip-art artifact removal, N = 15 for
 * texture smoothing, gamma = 5/255 .. 10/255. */
int ils_smooth_welsch(ils_plan* plan, const float* f, int H, int W, int C, float lambda, float gamma,
                      int N, float* out);

/* Detail enhancement (Sec. 4, the application the paper's figures show with
 * details boosted k = 3 times): out = u + k (f - u), u = u^N of ils_smooth.
 * The blend is fused into the final row pass (one extra read of f).
 * k finite; k = 0 gives ils_smooth, k = 1 gives f.  Other rules as
 * ils_smooth (out == f allowed). */
int ils_detail_enhance(ils_plan* plan, const float* f, int H, int W, int C, float lambda, float p,
                       float eps, int N, float k, float* out);

/* Luminance-only colour mode (Sec. 3.4, option (I)): for a planar RGB frame
 * (3 x H x W) smooth only Y = 0.299 R + 0.587 G + 0.114 B and add the change
 * of Y back to each channel, out_c = f_c + (v - Y) with v = u + k (Y - u)
 * (k = 0: plain smoothing; k > 0: detail enhancement of the luminance).
 * This is a YUV round trip that leaves U and V unchanged.  About a third of
 * the work of smoothing the three channels.  The workspace must hold
 * ils_luminance_workspace_bytes(H, W) (a plan for 3 channels always does).
 * out == f allowed. */
size_t ils_luminance_workspace_bytes(int max_H, int max_W);
int ils_smooth_luminance(ils_plan* plan, const float* f, int H, int W, float lambda, float p, float eps,
                         int N, float k, float* out);

/* Single-scale HDR tone mapping (Sec. 4, the application shown with p = 1,
 * lambda = 10): on a planar linear-radiance RGB frame f (3 x H x W, > 0),
 * L = log max(Y, 1e-6) with Y = 0.299 R + 0.587 G + 0.114 B; base B = u^N of
 * Algorithm 1 on L; detail D = L - B; L' = (B - max B) s + detail * D with
 * s = log(contrast) / (max B - min B) (s = 1 for a flat base); out_c =
 * f_c exp(L' - L), which keeps the colour ratios of every pixel.  The output
 * is linear (no display gamma) and not clipped.  contrast > 1, detail >= 0
 * finite.  Workspace as ils_smooth_luminance.  out == f allowed. */
int ils_tone_map(ils_plan* plan, const float* f, int H, int W, float lambda, float p, float eps, int N,
                 float contrast, float detail, float* out);

/* Multi-scale HDR tone mapping (Sec. 4.2, the multi-scale figure: p = 1,
 * lambda = 1/8, 1, 8).  L = log max(Y, 1e-6) as in ils_tone_map; K levels
 * B_k = u^N of Algorithm 1 on L with lambda = lambdas[k], each smoothed from
 * L itself (host array, increasing lambda expected but not required);
 * detail layers D_1 = L - B_1 and D_k = B_(k-1) - B_k; base B_K compressed
 * as in ils_tone_map (shifted to maximum 0, scaled to span log(contrast));
 * L' = compressed base + sum_k weights[k] D_k; out_c = f_c exp(L' - L).
 * With unit weights and the base's own range as contrast the log luminance
 * is kept up to a shift.  1 <= K <= ILS_MAX_SCALES; weights (host array)
 * finite and >= 0; contrast > 1.  The workspace must hold
 * ils_tone_map_multiscale_workspace_bytes(H, W, K) (the spectra of one
 * channel and K + 1 luminance planes).  out == f allowed. */
#define ILS_MAX_SCALES 4
size_t ils_tone_map_multiscale_workspace_bytes(int max_H, int max_W, int K);
int ils_tone_map_multiscale(ils_plan* plan, const float* f, int H, int W, const float* lambdas,
                            const float* weights, int K, float p, float eps, int N, float contrast, float* out);

/* Energy of Eq. (1), E(u) = sum (u - f)^2 + lambda sum (phi(D_x u) +
 * phi(D_y u)) over all pixels and channels, periodic differences, computed
 * in double: phi = (x^2 + eps)^(p/2) (Eq. (2)) for ils_energy, the Welsch
 * penalty 2 gamma^2 (1 - exp(-x^2 / (2 gamma^2))) (Eq. (18)) for
 * ils_energy_welsch.  f, u: device C x H x W float32; energy: device double,
 * written on the plan's stream.  For convergence studies (energy against the
 * iteration number). */
int ils_energy(ils_plan* plan, const float* f, const float* u, int H, int W, int C, float lambda, float p,
               float eps, double* energy);
int ils_energy_welsch(ils_plan* plan, const float* f, const float* u, int H, int W, int C, float lambda,
                      float gamma, double* energy);

/* As ils_smooth but starting from u^0 = u0 while the data term stays f
 * (N iterations of Eq. (7)-(9)).  With N = 1 this is the one-iteration map
 * T(u0) used to assess a candidate output by its fixed-point residual.
 * u0 may equal f; out must not overlap f or u0 unless out == f == u0. */
int ils_iterate_from(ils_plan* plan, const float* f, const float* u0, int H, int W, int C,
                     float lambda, float p, float eps, int N, float* out);

/* As ils_iterate_from with the constant c of Eqs. (3) and (11) given explicitly
 * instead of c = c0 = p eps^(p/2 - 1) (Sec. 3.3.3: any c >= c0 keeps the
 * energy decreasing; smaller c converges faster).  c < c0 (beyond a relative
 * 1e-6) is ILS_ERR_INVALID_ARG; c within a relative 1e-6 of c0 runs the
 * default c = c0 path exactly.  For convergence studies. */
int ils_iterate_from_c(ils_plan* plan, const float* f, const float* u0, int H, int W, int C, float lambda,
                       float p, float eps, float c, int N, float* out);

/* Smooth n frames of possibly different sizes and parameters in one
 * enqueue: frames of equal size, N and penalty form a class, run with one
 * launch per pass over a part of the class (one part per frame for frames
 * of one channel count with at least 4 Mi pixel-channels each, else two
 * parts); the parts form two independent chains of passes, the whole
 * sequence replayed as one HIP graph (unless ILS_PLAN_NO_GRAPH or pass
 * timing is active).  Results are bitwise those of one ils_smooth (or
 * ils_iterate_from, when u0 is set) per frame.  frames is a host array,
 * read during the call.  Each frame obeys the rules of ils_smooth.  Returns
 * ILS_ERR_INVALID_ARG for n above the plan's max_frames and
 * ILS_ERR_WORKSPACE when the workspace holds less than
 * ils_batch_workspace_bytes(frames, n), before anything is enqueued. */
int ils_smooth_batch(ils_plan* plan, const ils_frame* frames, int n);

/* Per-frame root-mean-square difference: rms[i] = sqrt(mean((a_i - b_i)^2))
 * over the count[i] floats of frame i.  a, b, count: host arrays of n device
 * pointers / counts; rms: device float[n].  Used for the fixed-point
 * residual of a candidate output. */
int ils_rms_diff(ils_plan* plan, const float* const* a, const float* const* b,
                 const long long* count, int n, float* rms);

/* Pass timing.  Between ils_profile_begin and ils_profile_end every pass
 * launch the plan enqueues is bracketed by two HIP events on the plan's
 * stream.  ils_profile_end synchronises on the last event and writes, per
 * pass kind k (0 = first row pass, 1 = middle row pass, 2 = final row pass,
 * 3 = column pass), the summed duration total_ms[k] and the launch count
 * count[k] (host arrays of 4).  Timing adds two event records per launch. */
int ils_profile_begin(ils_plan* plan);
int ils_profile_end(ils_plan* plan, double* total_ms, int* count);

/* Enqueue ONE launch of one pass kind of the sequence ils_smooth runs for
 * this frame (kind 0 = first row pass with u^0 = f, 1 = middle row pass,
 * 2 = final row pass, 3 = column pass; Alg. 1 with the solve of Eq. (9)),
 * with the frame's tuned tile shapes, on the plan's workspace spectra: the
 * row passes read the second half spectrum (and f), the column pass reads
 * the first; the final pass writes out (C x H x W, device).  The spectra's
 * contents are left meaningless.  For timing a pass on its own with events
 * around a run of calls (no bracketing of each launch); other rules as
 * ils_smooth. */
int ils_enqueue_pass(ils_plan* plan, int kind, const float* f, float* out, int H, int W, int C, float lambda,
                     float p, float eps);

/* Last asynchronous HIP error seen by the plan (ILS_OK if none); clears it. */
int ils_last_error(ils_plan* plan);

/* ---- tile shapes (the autotuner) ----
 * Transform lengths of 480 and more are compiled with up to six row-band
 * heights (rows per workgroup of the row passes) and up to four column-tile
 * widths (spectrum columns per workgroup of the column pass).  Every shape runs the
 * same arithmetic on every row and column, so the results are bitwise equal;
 * only the speed differs.  The first smoothing call for a size H x W x C
 * times the shapes on the plan's stream (a few launches on workspace data,
 * one host synchronisation) and keeps the faster ones for the plan's life.
 * A call made while the stream is being captured into a graph keeps the
 * default shapes and leaves the size untuned.  A row shape's height is the
 * most rows a workgroup holds: a single frame's rows are cut into balanced
 * bands of at most that many rows, as many as fill whole rounds of the
 * compute units.  In ils_smooth_batch, frames large enough to be parts of
 * their own take the widest column tile.  Environment: ILS_TUNE=0
 * keeps the defaults; ILS_TUNE_CACHE=<file> reads earlier choices at plan
 * creation ("arch H W C rows-per-band columns-per-tile" per line) and
 * appends new ones.
 *
 * ils_shape_variants: number of row / column shapes for a supported size
 *   (1 to 6 and 1 to 4; 1 and 1 for a frame on the runtime-length passes).
 *   ILS_ERR_UNSUPPORTED_SIZE otherwise.
 * ils_plan_tune: tune the size now if it is not yet (synchronises the
 *   plan's stream) and return the chosen shape indices (0 = default).
 * ils_plan_set_shapes: fix the shapes for a size (indices below the counts
 *   of ils_shape_variants, else ILS_ERR_INVALID_ARG); no GPU work. */
int ils_shape_variants(int H, int W, int* n_row, int* n_col);
int ils_plan_tune(ils_plan* plan, int H, int W, int C, int* row_shape, int* col_shape);
int ils_plan_set_shapes(ils_plan* plan, int H, int W, int C, int row_shape, int col_shape);

/* ---- allocation-free smoothing ----
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * computation of ils_smooth (Algorithm 1, no plan, default tile shapes)
 * with its two half spectra in a file-scope device array of the library
 * (64 MiB per GPU, held from the library's loading until the process ends)
 * instead of a caller workspace (its first 4 MiB hold the transform tables
 * of every supported length).  The first call on a device copies the tables
 * into that array synchronously; later calls only enqueue on hip_stream.
 * No call allocates or frees memory.
 *   f, out : device pointers, C x H x W float32 (out == f allowed).
 *   Frames whose two half spectra exceed ils_noalloc_max_bytes()
 *   (2 * C * H * (W/2+1 rounded up to 16) * 8 bytes; a 1920 x 1080 RGB
 *   frame fits, a 3840 x 2160 RGB frame does not) return ILS_ERR_WORKSPACE
 *   before anything is enqueued.  Other rules and results as ils_smooth.
 * Every call on one GPU uses the same array: calls that overlap on one GPU
 * (other streams, other host threads) race and give undefined results. */
size_t ils_noalloc_max_bytes(void);
int ils_smooth_noalloc(const float* f, int H, int W, int C, float lambda, float p, float eps, int N, float* out,
                       void* hip_stream);

/* Destroy a plan (NULL is accepted).  Does not free the workspace. */
int ils_plan_destroy(ils_plan* plan);

/* ---- single-pass entry points (stage checks; same validation rules) ----
 * spec: device complex64 array C x H x (W/2+1), interleaved (re, im).
 * ils_debug_rhs_spectrum : spec = 2 * rfft along rows of
 *     r = f + (lambda c / 2) D^T mu(u0),  mu = mu_paper / c      (Eq. (7), (9))
 * ils_debug_column_solve : spec_out = column FFT, divide by
 *     2 H W (1 + (lambda c / 2)(4 sin^2(pi kx/W) + 4 sin^2(pi ky/H))), column
 *     inverse FFT (unnormalised), applied to spec_in
 * ils_debug_row_inverse  : out = unnormalised inverse real FFT along rows of
 *     spec (imaginary parts of the DC and Nyquist bins ignored). */
int ils_debug_rhs_spectrum(ils_plan* plan, const float* f, const float* u0, int H, int W, int C,
                           float lambda, float p, float eps, float* spec);
int ils_debug_column_solve(ils_plan* plan, const float* spec_in, int H, int W, int C,
                           float lambda, float p, float eps, float* spec_out);
int ils_debug_row_inverse(ils_plan* plan, const float* spec, int H, int W, int C, float* out);

#ifdef __cplusplus
}
#endif

#endif /* ILS_H_ */
