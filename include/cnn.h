/*
 * cnn.h - C ABI of the learned warm start for the SR Split Bregman solver.
 *
 * A 4-level encoder-decoder network (3x3 convolutions with zero padding,
 * 16 -> 32 -> 64 -> 128 channels, two per level, ReLU, 2x2 average pooling,
 * nearest upsampling + 3x3 convolution, concatenated skips, 1x1 head) maps
 * (image f, edge map g, initial level set phi^0) to a predicted level set
 * phi-hat, which sr_set_state then hands to the Split Bregman iteration
 * (Algorithm 1 of the paper refines it and judges the result).
 *
 * Activations and weights are BF16, products accumulate in FP32 on the
 * MFMA units (v_mfma_f32_16x16x16_bf16); gradients, master weights and the
 * Adam moments are FP32.  Every kernel is the library's own.
 *
 * Conventions: device pointers; images are [n][H][W] float32 (n <= batch);
 * H and W are multiples of 32 in [32, 2048] (every level's pixel count is
 * then a multiple of 16, one MFMA tile) and batch*H*W <= 2^26.  The caller allocates the
 * workspace (cnn_workspace_size) and owns it; the library never allocates
 * device memory.  Calls enqueue on the stream given to cnn_create; calls
 * returning host values synchronise it.  Return codes are those of sr.h
 * (0 = OK, < 0 error; cnn_last_error describes the last error).
 *
 * The flat parameter vector lists, for each layer in the order
 * L0a L0b L1a L1b L2a L2b L3a L3b U2 D2 U1 D1 U0 D0 head, its weights
 * [cout][cin][3][3] (head: [1][16]) followed by its biases [cout].
 */
#ifndef CNN_H_
#define CNN_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cnn_ctx cnn_ctx;

/* Number of float parameters of the network. */
int cnn_num_params(int64_t* n);

/* Workspace bytes for training / inference on up to `batch` images of H x W. */
int cnn_workspace_size(int32_t batch, int32_t H, int32_t W, size_t* bytes);

int cnn_create(cnn_ctx** out, int32_t batch, int32_t H, int32_t W, void* workspace, size_t bytes,
               void* hip_stream);

/* Load / read the flat FP32 parameter vector (device pointer).  Loading
 * resets the Adam moments and step count. */
int cnn_set_params(cnn_ctx* ctx, const float* params);
int cnn_get_params(cnn_ctx* ctx, float* params);

/* Forward pass on n images: input channels (f, g, clip(phi0, +-clip)/clip)
 * in BF16; phi_pred = clip * head output.  phi_pred may be NULL (training). */
int cnn_forward(cnn_ctx* ctx, const float* f, const float* g, const float* phi0, int32_t n, float clip,
                float* phi_pred);

/* Copy a stored tensor of the last cnn_forward, converted to FP32, to out
 * (device, channels-last [n][H_l][W_l][C]): which = 0..13 the ReLU output of
 * the 3x3 layer of that index (order of the parameter vector), 14 the
 * network input (C = 4, the 4th channel zero), 15 the head output (C = 1),
 * 16..18 the pooled skips entering levels 1..3; after a cnn_backward,
 * 19..32 the masked BF16 output gradient of 3x3 layer which-19 (C = its
 * output channels).  For inspection and tests. */
int cnn_get_activation(cnn_ctx* ctx, int32_t which, float* out);

/* Backward pass for the images of the last cnn_forward: loss = mean over
 * pixels of (head - clip(target, +-clip)/clip)^2, gradients of every
 * parameter accumulated afresh.  *loss receives the loss (synchronises);
 * grad_out (nullable, device) receives the flat FP32 gradient. */
int cnn_backward(cnn_ctx* ctx, const float* target, float clip, double* loss, float* grad_out);

/* One Adam step on the gradients of the last cnn_backward (bias-corrected
 * moments), then the BF16 weight copies are refreshed. */
int cnn_adam_step(cnn_ctx* ctx, float lr, float beta1, float beta2, float eps);

void cnn_destroy(cnn_ctx* ctx);
const char* cnn_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* CNN_H_ */
