/*
 * nsim_up.h -- C ABI of the learned temporal upsampler (libnsim_up.so).
 *
 * Purpose (paper Sec. 1, contribution on efficient high-fidelity event
 * simulation; Sec. 2, event-camera paragraph): event simulation wants
 * frames at 1000 FPS or more, since distant frames let crossings alias or go
 * missing.  This library predicts the seven log-intensity frames between
 * two log frames L0, L8 that are eight frame intervals apart, so the event
 * generator (nsim_ev_step_log) can run at the full rate on frames rendered
 * at one eighth of it.
 *
 * Network (fixed): a 3-level U-Net, two 3x3 convolutions with bias and ReLU
 * per level (16, 32, 64 channels at full, half, quarter resolution), 2x2
 * average pooling down, nearest 2x upsampling up with the encoder's skip
 * tensor concatenated first (96 -> 32, 32 -> 32 at half, 48 -> 16, 16 -> 16
 * at full resolution), a 1x1 head 16 -> 7 giving residuals:
 *   L_j = (1 - j/8) L0 + (j/8) L8 + delta_j,  j = 1..7.
 * bfloat16 weights and activations, FP32 accumulation on the matrix cores,
 * FP32 master weights and Adam (beta1 0.9, beta2 0.999, eps 1e-8); loss is
 * the mean absolute error over the predicted log frames.
 *
 * Parameters (FP32, count nsim_up_num_params) are one flat array in this
 * order: for each convolution e1a, e1b, e2a, e2b, e3a, e3b, d2a, d2b, d1a,
 * d1b its weights [C_out][3][3][C_in] then its bias [C_out]; then the head
 * weights [7][16] and bias [7].
 *
 * Memory: "device" pointers are HIP device memory owned by the caller;
 * frames are planar FP32 [N][H][W] (predictions [N][7][H][W]).  Every call
 * is enqueued on the handle's stream and returns without synchronising.
 * H and W must be multiples of 4 and N*H*W at most the configured maximum.
 * Errors: NSIM_UP_OK (0) or a negative code; nsim_up_last_error() gives
 * the message.  A handle is not thread-safe.
 */
#ifndef NSIM_UP_H
#define NSIM_UP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NSIM_UP_OK 0
#define NSIM_UP_EINVAL (-1)
#define NSIM_UP_ENOMEM (-2)
#define NSIM_UP_EHIP (-4)

typedef struct nsim_up nsim_up_t;

typedef struct nsim_up_config {
    int64_t max_pixels;   /* largest N*H*W of any call, 16 to 2^30
                             (else NSIM_UP_EINVAL); a call with more
                             pixels fails with NSIM_UP_EINVAL */
    uint64_t seed;        /* weight initialisation (He-uniform, zero
                             biases, zero head) */
} nsim_up_config;

int nsim_up_create(const nsim_up_config* cfg, void* stream, nsim_up_t** out);
int nsim_up_destroy(nsim_up_t* h);
const char* nsim_up_last_error(const nsim_up_t* h);

int64_t nsim_up_num_params(const nsim_up_t* h);
/* Copy the FP32 master parameters out (device dst) or in (device src; also
 * clears the Adam moments and step count). */
int nsim_up_get_params(nsim_up_t* h, float* dst, int64_t n);
int nsim_up_set_params(nsim_up_t* h, const float* src, int64_t n);

/* Predict the 7 intermediate log frames (device out [N][7][H][W]). */
int nsim_up_forward(nsim_up_t* h, const float* L0, const float* L8, int32_t N,
                    int32_t H, int32_t W, float* out);

/* Forward, L1 loss against target [N][7][H][W] and the gradient of every
 * parameter (kept in the handle).  pred (device [N][7][H][W]) and loss
 * (device scalar) may be NULL. */
int nsim_up_backward(nsim_up_t* h, const float* L0, const float* L8,
                     const float* target, int32_t N, int32_t H, int32_t W,
                     float* pred, float* loss);
/* Copy the last gradients out (device dst, parameter order above). */
int nsim_up_get_grads(nsim_up_t* h, float* dst, int64_t n);
/* One Adam update of the master weights from the last gradients. */
int nsim_up_adam_step(nsim_up_t* h, float lr);
/* nsim_up_backward followed by nsim_up_adam_step. */
int nsim_up_train_step(nsim_up_t* h, const float* L0, const float* L8,
                       const float* target, int32_t N, int32_t H, int32_t W,
                       float lr, float* loss);

/* L[i] = ln(I[i] + eps) in FP32 for n device floats (the event model's log,
 * paper Sec. 2 event-camera paragraph), on `stream`. */
int nsim_up_log_frames(const float* I, float* L, int64_t n, float eps,
                       void* stream);

/* Diagnostic: C = A B for 16x16 bfloat16 row-major A, B (device) with one
 * matrix-core instruction, C 16x16 FP32 row-major (device). */
int nsim_up_diag_mfma(const uint16_t* A, const uint16_t* B, float* C,
                      void* stream);

/* Diagnostic: C = A B for A 16x32 and B 32x16 bfloat16 row-major (device)
 * with one 16x16x32 matrix-core instruction (gfx950), C 16x16 FP32
 * row-major (device). */
int nsim_up_diag_mfma32(const uint16_t* A, const uint16_t* B, float* C,
                        void* stream);

#ifdef __cplusplus
}
#endif
#endif /* NSIM_UP_H */
