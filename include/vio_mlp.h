/*
 * vio_mlp.h -- the learned-initialisation network of the frontend, on gfx950.
 *
 * A project addition (the paper initialises each track from the backend's
 * prediction, Sec. III-E): a multilayer perceptron maps 32 features of a
 * keypoint -- the previous flows of its 8 nearest neighbours and a 4x4-pooled
 * patch -- to a displacement guess and a confidence:
 *   h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), y = W3 h2 + b3,
 *   W1 128x32, W2 128x128, W3 3x128; guess (16 y0, 16 y1) px, confidence
 *   sigmoid(y2).
 * The matrix products run on BF16 MFMA with FP32 accumulation: inputs, weights
 * and the post-ReLU activations are rounded to bfloat16 (nearest even);
 * biases, sums and the FP32 master weights stay in float. Training minimises
 * Huber (delta 1 px) on the guess against a target displacement plus binary
 * cross-entropy of y2 against [|guess - target| <= 2 px], averaged over the
 * batch, with Adam on the master weights.
 *
 * Parameter vector (float, VIO_MLP_NPARAM entries, row-major): W1[128][32],
 * b1[128], W2[128][128], b2[128], W3[3][128], b3[3].
 *
 * Errors: VIO_OK or a negative vio_result (vio_frontend.h). Device pointers
 * are borrowed for the call; work is queued on `hip_stream` (a hipStream_t,
 * NULL = the legacy default stream) and the call returns without waiting
 * unless stated.
 */
#ifndef VIO_MLP_H
#define VIO_MLP_H

#include <stdint.h>

#include "vio_frontend.h"

#ifdef __cplusplus
extern "C" {
#endif

#define VIO_MLP_IN 32
#define VIO_MLP_HIDDEN 128
#define VIO_MLP_OUT 3
#define VIO_MLP_NPARAM 21123

typedef struct vio_mlp vio_mlp;

/* Allocates the model (master weights, bfloat16 copies, Adam moments) and the
 * training scratch for batches of up to max_batch rows (1..65536). */
int vio_mlp_create(int32_t max_batch, vio_mlp** out);
void vio_mlp_destroy(vio_mlp* m);

/* Copies host parameters in (n must be VIO_MLP_NPARAM) and resets Adam. Waits. */
int vio_mlp_set_params(vio_mlp* m, const float* params, int32_t n);
/* Copies the master parameters out (n >= VIO_MLP_NPARAM). Waits. */
int vio_mlp_get_params(vio_mlp* m, float* params, int32_t n);

/* y[k][3] = network(x[k][32]) for k rows (device pointers, float). */
int vio_mlp_forward(vio_mlp* m, const float* d_x, int32_t k, float* d_y, void* hip_stream);

/* Loss and gradient of a batch (k <= max_batch rows, targets[k][2] px):
 * d_grad receives VIO_MLP_NPARAM floats (device); *loss (host) the batch loss.
 * Waits for the result. */
int vio_mlp_gradient(vio_mlp* m, const float* d_x, const float* d_targets, int32_t k, float* d_grad, float* loss,
                     void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * results as vio_mlp_gradient (bit for bit), with the training scratch (the
 * transposed bfloat16 operands, the output and loss gradients, the loss) in a
 * device array the library holds, one per GPU, for the life of the process
 * (VIO_MLP_NOALLOC_MAX_ROWS rows, about 4.4 MB), instead of the handle's
 * buffers; k may exceed the handle's max_batch up to that maximum. Allocates
 * nothing (no hipMalloc, hipFree or allocating library call); the first call
 * on a device looks the array's address up. Every call on a GPU shares that
 * GPU's array: calls that overlap on one GPU (on different streams or
 * threads) race and must be serialised by the caller. Waits for the result
 * like vio_mlp_gradient. Errors: VIO_EINVAL for a null pointer, k < 1 or
 * k > VIO_MLP_NOALLOC_MAX_ROWS; VIO_EDEVICE. */
#define VIO_MLP_NOALLOC_MAX_ROWS 4096
int vio_mlp_gradient_noalloc(vio_mlp* m, const float* d_x, const float* d_targets, int32_t k, float* d_grad,
                             float* loss, void* hip_stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on the batch's gradient;
 * *loss (host, may be NULL) receives the batch loss before the step. Waits
 * when loss is not NULL. */
int vio_mlp_train_step(vio_mlp* m, const float* d_x, const float* d_targets, int32_t k, float lr, float* loss,
                       void* hip_stream);

/* Installs trained parameters in a frontend created with init_mode =
 * VIO_INIT_LEARNED; rho replaces params.learned_rho when >= 0. Waits. */
int vio_frontend_set_mlp(vio_frontend* h, const float* params, int32_t n, float rho);

/* Diagnostics: the network inputs of camera `camera`'s previous keypoints
 * computed in the last frame (one row of VIO_MLP_IN floats per temporal
 * record, in record order); *n_out = rows. Learned mode only. */
int vio_frontend_get_features(vio_frontend* h, int32_t stream, int32_t camera, float* out, int32_t capacity,
                              int32_t* n_out);

#ifdef __cplusplus
}
#endif

#endif /* VIO_MLP_H */
