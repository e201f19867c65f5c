/*
 * ils_net.h -- C ABI of the learned surrogate of ILS smoothing (not part of
 * the paper; the paper's own method is in ils.h).
 *
 * Network: six 3x3 convolutions with periodic padding, 32 channels, ReLU
 * after the first five; input = RGB image + constant lambda and p maps;
 * output v = f + z6 (the network predicts the correction to the image).
 * Weights and activations are bf16 with fp32 accumulation on the MFMA
 * units; master weights and Adam moments are fp32.  Images are planar
 * float32 (B, 3, H, W), contiguous, device pointers owned by the caller.
 * All calls enqueue on the network's stream and return after enqueue,
 * except ils_net_set_state / ils_net_get_state (synchronous) and
 * ils_surrogate_infer (synchronises once to read the residuals).  The
 * activations, gradients and optimiser state live in the network's
 * workspace and are shared by all its calls, so calls on one network must
 * not overlap (keep them on its stream, from one host thread at a time).
 *
 * Parameter layout (fp32, ils_net_param_count() values): for each layer in
 * order, w[co][ci][3][3] then b[co]; layers 5->32, 32->32 (x4), 32->3.
 * Convolution: z[co][y][x] = b[co] + sum w[co][ci][a][c] x[ci][(y+a-1) mod H][(x+c-1) mod W].
 */
#ifndef ILS_NET_H_
#define ILS_NET_H_

#include <stddef.h>

#include "ils.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ils_net ils_net;

/* Number of fp32 parameters. */
int ils_net_param_count(void);

/* Device workspace bytes for batches up to max_B images of max_H x max_W
 * (activations, gradients, parameters, optimiser state).  0 if invalid. */
size_t ils_net_workspace_bytes(int max_B, int max_H, int max_W);

/* Create a network on caller-owned workspace (256-byte aligned, at least
 * ils_net_workspace_bytes).  Parameters are undefined until set_state. */
int ils_net_create(ils_net** net, int max_B, int max_H, int max_W, void* workspace, size_t ws_bytes,
                   void* hip_stream);
int ils_net_set_stream(ils_net* net, void* hip_stream);

/* Host copies of the state.  m, v may be NULL (zeros on set, skipped on get). */
int ils_net_set_state(ils_net* net, const float* params, const float* m, const float* v, long long step);
int ils_net_get_state(ils_net* net, float* params, float* m, float* v, long long* step);

/* v = network(f, lambda, p).  lam, p: device float[B] (one value per image). */
int ils_net_forward(ils_net* net, const float* f, const float* lam, const float* p, int B, int H, int W,
                    float* v);

/* Gradients of the mean squared error between network(f) and target, in
 * the parameter layout (device float[param_count]); loss: device float[1].
 * Parameters are not changed. */
int ils_net_gradients(ils_net* net, const float* f, const float* lam, const float* p, const float* target,
                      int B, int H, int W, float* grad, float* loss);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) on the
 * mean squared error against target.  loss (device float[1]) may be NULL. */
int ils_net_train_step(ils_net* net, const float* f, const float* lam, const float* p, const float* target,
                       int B, int H, int W, float lr, float* loss);

int ils_net_last_error(ils_net* net);
int ils_net_destroy(ils_net* net);

/* Residual-gated inference for B RGB images of H x W.
 *   v = network(f) is written to out; for each image the map T (one ILS
 *   iteration, Eqs. (7)-(9), from u^0 = v with data term f) gives the
 *   fixed-point residual R = rms(T(v) - v) over the image's 3HW values;
 *   images with R > tau (or a non-finite R) are recomputed by plain ILS with
 *   N iterations into out.
 *   lam_dev/p_dev: device float[B]; lam_host/p_host: the same values on the
 *   host; tv_scratch: device float[B*3*H*W]; residual_host: float[B];
 *   fallback_host: int[B] (1 where plain ILS was used).
 *   tau must be finite (ILS_ERR_NOT_CALIBRATED otherwise).  T(v) and the
 *   fallback run as batched calls when the plan holds B frames of this size
 *   (else image by image, with the same result).  The plan enqueues on the
 *   network's stream during the call; its own stream is restored before
 *   the call returns. */
int ils_surrogate_infer(ils_net* net, ils_plan* plan, const float* f, const float* lam_dev, const float* p_dev,
                        const float* lam_host, const float* p_host, float eps, int N, int B, int H, int W,
                        float tau, float* out, float* tv_scratch, float* residual_host, int* fallback_host);

/* The same gate for a list of frames of uneven sizes (a host array of
 * nframes descriptors, 1 <= nframes <= max_B, each an RGB image within the
 * network's max_H x max_W): frames[i].f is the input, frames[i].out
 * receives the network output, replaced by plain ILS with frames[i].N
 * iterations (frames[i].lambda, p, eps) where the frame's fixed-point
 * residual exceeds tau.  Each frame needs C = 3, the generalised
 * Charbonnier penalty and u0 = NULL (or f); anything else is
 * ILS_ERR_INVALID_ARG and nothing is enqueued.  tv_scratch: device float
 * array of sum_i 3 H_i W_i values (the frames' T(v) in list order);
 * residual_host: float[nframes]; fallback_host: int[nframes].  The network
 * runs frame by frame; T(v) and the fallback are one batched call each when
 * the plan holds the frames (else frame by frame).  Per frame the results
 * are bitwise those of ils_surrogate_infer.  Synchronises once, like it. */
int ils_surrogate_infer_frames(ils_net* net, ils_plan* plan, const ils_frame* frames, int nframes, float tau,
                               float* tv_scratch, float* residual_host, int* fallback_host);

#ifdef __cplusplus
}
#endif

#endif /* ILS_NET_H_ */
