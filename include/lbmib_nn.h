/*
 * lbmib_nn.h -- C ABI of the neural operator of the learned warm start (same library as lbmib.h).
 *
 * The paper solves each steady problem by time marching from a uniform state (Sec. 2.5). This
 * part predicts the steady fields (rho, u_x, u_y, T) of a 2D body in a uniform stream from a
 * signed-distance field and the flow parameters, so that the marching can start close to the
 * steady state (a warm start); the plain method then runs to convergence from it, stays the
 * fallback when the prediction is unusable, and measures its error.
 *
 * The network is a five-level convolutional U-Net (channels 32, 64, 128, 256, 256; 3x3
 * convolutions with ReLU, 2x2 average pooling, nearest 2x upsampling with skip concatenation,
 * a 1x1 head), on NHWC activations in bf16 with FP32 accumulation on the matrix cores, FP32
 * master parameters and an Adam update. Images are batch x H x W pixels with pixel
 * (n, y, x) at index (n H + y) W + x; input planes [P][4] and outputs/targets [P][4] are FP32.
 *
 * Conventions as in lbmib.h: 0 on success, negative codes on error, the last error message of a
 * handle from nn_unet_last_error; all work is ordered on the stream given at creation; the caller
 * owns the device workspace (it must outlive the handle); the library allocates no device memory.
 */
#ifndef LBMIB_NN_H
#define LBMIB_NN_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { NN_OK = 0, NN_E_INVAL = -1, NN_E_NOMEM = -2, NN_E_HIP = -3, NN_E_STATE = -4 };

typedef struct nn_unet nn_unet;

/* Number of FP32 parameters. Flat layout, layer by layer in the order encoder levels 0..3
 * (two convolutions each), bottleneck (two), decoder levels 3..0 (two each), head: for each
 * layer the weights [cout][taps][cin] (tap = 3 (dy + 1) + (dx + 1)), then the biases [cout].
 * The first layer has cin = 8 (the 4 input planes and 4 zero planes). */
long long nn_unet_param_count(void);

/* Workspace bytes for a batch capacity and image size (0 if invalid: H % 16 or W % 128 != 0). */
size_t nn_unet_workspace_bytes(int batch, int H, int W);

/* Create a network; parameters start at zero. Errors: NN_E_INVAL, NN_E_NOMEM, NN_E_HIP. */
int nn_unet_create(int batch, int H, int W, void* dev_workspace, size_t bytes, void* hip_stream, nn_unet** out);

/* Set / read the FP32 parameters (host or device array of nn_unet_param_count floats).
 * Setting also clears the Adam moments. Host transfers synchronise. */
int nn_unet_set_params(nn_unet* u, const float* params, int on_device);
int nn_unet_get_params(nn_unet* u, float* params, int on_device);

/* Gradient of the loss of the last backward pass with respect to the parameters (flat layout). */
int nn_unet_get_grads(nn_unet* u, float* grads, int on_device);

/* Forward pass of b <= batch images: d_in [b H W][4] -> d_out [b H W][4] (device, FP32; d_out
 * may be NULL). Keeps the activations for nn_unet_backward. Asynchronous. */
int nn_unet_forward(nn_unet* u, int b, const float* d_in, float* d_out);

/* Backward pass of the masked mean squared error L = sum_p m_p |out_p - t_p|^2 / (4 sum_p m_p)
 * of the last forward: d_target [b H W][4], d_mask [b H W] (NULL = all ones), device FP32.
 * Writes the parameter gradient; d_loss (device, nullable) receives {L, 4 sum m} in FP64.
 * Errors: NN_E_STATE before any forward pass. Asynchronous. */
int nn_unet_backward(nn_unet* u, const float* d_target, const float* d_mask, double* d_loss);

/* One Adam step with bias correction at step t >= 1 and decoupled weight decay:
 * theta -= lr (m^ / (sqrt(v^) + eps) + weight_decay theta). Asynchronous. */
int nn_unet_adam(nn_unet* u, double lr, double beta1, double beta2, double eps, int t, double weight_decay);

/* Clipping by the global L2 norm of the parameter gradient of the last backward pass:
 * g *= min(1, max_norm / ||g||_2), with ||g||_2 summed in FP64 in a fixed order. d_norm (device,
 * nullable) receives {||g||_2, applied scale}. Runs on the stream without host synchronisation.
 * Errors: NN_E_INVAL for max_norm <= 0. Asynchronous. */
int nn_unet_clip_grad_norm(nn_unet* u, double max_norm, double* d_norm);

void nn_unet_destroy(nn_unet* u);
const char* nn_unet_last_error(nn_unet* u);

#ifdef __cplusplus
}
#endif
#endif /* LBMIB_NN_H */
