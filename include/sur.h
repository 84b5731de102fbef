/*
 * sur.h -- C ABI of the learned surrogate of the IMPM sensor (in libimpm.so).
 *
 * The surrogate predicts one frame of the elastomer simulation of arXiv
 * 2405.02914 (Sec. III-A: the surface displacement that IMPM produces when the
 * indenter moves between two height-map frames, Sec. IV-B) so that a serving
 * loop can skip most IMPM solves and fall back to the simulator to re-anchor.
 * The paper itself has no learned component; the method is the reference the
 * surrogate's error is measured against.
 *
 * Network (U-shape, NHWC BF16 activations and weights, FP32 accumulation on
 * the MFMA units, FP32 master weights):
 *   level 0 (H x W, c0 ch)  conv0 in->c0, conv1 c0->c0               skip s0 = a1
 *   level 1 (H/2, c1)       conv2 c0->c1 stride 2, conv3 c1->c1       skip s1 = a3
 *   level 2 (H/4, c2)       conv4 stride 2, conv5                     skip s2 = a5
 *   level 3 (H/8, c3)       conv6 stride 2, conv7
 *   decoder                 conv8  = conv(up2(a7)) + s2, conv9
 *                           conv10 = conv(up2(a9)) + s1, conv11
 *                           conv12 = conv(up2(a11)) + s0, conv13
 *   head                    next = prev + (a13 W_h^T + b_h)   (1x1, FP32 out)
 * All convolutions are 3x3 with zero padding 1, bias and ReLU; up2 repeats
 * each pixel 2 x 2.
 *
 * Inputs, per sample (all FP32, device memory, row-major):
 *   depth_mm  H x W      depth of the indenter below the slab top (mm); the
 *                        network sees it clipped to [-3, 3]
 *   pose6     6          pose change since the previous frame: translation
 *                        (mm) and rotation vector (rad)
 *   prev_mm   H x W x 3  previous surface displacement (mm)
 * Output: next_mm H x W x 3 (mm).
 *
 * Parameters (sur_get_params / sur_set_params, FP32 flat): for conv0..conv13
 * W[Cout][3][3][Cin] then b[Cout] (Cin of conv0 = in_ch = 10), then the head
 * W_h[3][c0] and b_h[3].
 *
 * Training (sur_train_step): loss = mean over samples, pixels and components
 * of (next - target)^2; gradients by backpropagation with pre-activation
 * gradients stored in BF16; Adam (Kingma and Ba 2015) with bias correction on
 * the FP32 master weights, which are then rounded to BF16 for the next step.
 *
 * Ownership and errors as in impm.h: the handle owns its device memory; input
 * and output pointers belong to the caller; calls return SUR_OK (0) or a
 * negative code, sur_last_error holds the message.  All work is enqueued on
 * the handle's stream; sur_train_step returns after enqueueing unless a loss
 * is requested.  Not thread-safe per handle.
 */
#ifndef SUR_H
#define SUR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { SUR_OK = 0, SUR_EINVAL = -1, SUR_ENOMEM = -2, SUR_EHIP = -3, SUR_EIO = -4 };

typedef struct {
    int32_t H, W;              /* image size, multiples of 8 */
    int32_t channels[4];       /* c0..c3, each 32, 64, 128 or 256, c0 <= 64 (default 32, 64, 128, 256) */
    int32_t max_batch;         /* largest n of any call */
    int32_t _pad0;
    uint64_t seed;             /* He-normal initial weights (SplitMix64 + Box-Muller) */
    float lr, beta1, beta2, eps;   /* Adam */
} sur_params;

typedef struct sur_s sur_t;

/* 128 x 128, channels 32-64-128-256, batch 64, Adam(1e-3, 0.9, 0.999, 1e-8). */
int sur_params_default(sur_params* p);
int sur_create(const sur_params* p, void* hip_stream, sur_t** out);
void sur_destroy(sur_t* s);
int sur_num_params(const sur_t* s, int64_t* n);

/* next_mm = network(depth, pose, prev) for n samples (device pointers). */
int sur_infer(sur_t* s, const float* depth_mm, const float* pose6, const float* prev_mm, float* next_mm,
              int32_t n);

/* One Adam step on n samples (device pointers).  loss_out (host, may be NULL):
 * the batch loss before the update; requesting it synchronises the stream. */
int sur_train_step(sur_t* s, const float* depth_mm, const float* pose6, const float* prev_mm,
                   const float* target_mm, int32_t n, float* loss_out);

/* Contact area of n samples (device pointers): area[i] = number of pixels of
 * sample i with depth_mm + disp_mm[..., 2] >= -tol_mm, i.e. where the
 * indenter's lower surface is within tol of the displaced elastomer surface
 * or below it.  The serving loop's trigger for an IMPM re-solve. */
int sur_contact_area(sur_t* s, const float* depth_mm, const float* disp_mm, int32_t n, float tol_mm, float* area);

/* Learning rate of the following Adam steps (a schedule is the caller's). */
int sur_set_lr(sur_t* s, float lr);

/* Same as sur_train_step without the update: leaves the gradients for
 * sur_get_grads (n_params floats, layout of sur_get_params). */
int sur_compute_grads(sur_t* s, const float* depth_mm, const float* pose6, const float* prev_mm,
                      const float* target_mm, int32_t n, float* loss_out);
int sur_get_grads(sur_t* s, float* out_host);

/* FP32 master parameters (host memory, n_params floats); set also resets the
 * Adam moments and step count. */
int sur_get_params(sur_t* s, float* out_host);
int sur_set_params(sur_t* s, const float* in_host);

/* Parameters and Adam state to / from a file (little-endian binary with a
 * header naming the sizes). */
int sur_save(sur_t* s, const char* path);
int sur_load(sur_t* s, const char* path);

/* Parity hooks: BF16 bits (host memory) of convolution `layer`'s activation
 * (which = 0, after the last forward pass) or of its pre-activation gradient
 * (which = 1, after the last backward pass), n_last x h x w x c of that layer
 * where n_last is the batch of the last call.  which = 2: the network input
 * (n_last x H x W x 32, channels 10..31 zero). */
int sur_debug_read(sur_t* s, int32_t which, int32_t layer, uint16_t* out_host);

const char* sur_last_error(const sur_t* s);

#ifdef __cplusplus
}
#endif

#endif /* SUR_H */
