/*
 * wsnet.h -- C ABI of the learned warm start: a convolutional U-Net whose
 * forward and backward passes run on hand-written BF16 MFMA kernels (gfx950)
 * with FP32 accumulation, trained with mean-squared error and Adam on FP32
 * master parameters.
 *
 * The lattice Boltzmann paper has no learned component; the network maps a
 * channel's initial condition (phase field, pressure-gradient plane, NCI
 * strength plane) to a predicted steady phase and velocity field, from which
 * the lattice Boltzmann run is started (the steady emulsion flows of the
 * Results section are what it is trained on).
 *
 * Architecture (levels L, base channels C0, C_l = C0 * 2^l, image H x W):
 *   encoder l = 0..L-1: 3x3 conv + ReLU (in -> C_l), 3x3 conv + ReLU,
 *                       2x2 max pool (l < L-1);
 *   decoder l = L-2..0: 2x2 stride-2 transposed conv (C_{l+1} -> C_l),
 *                       concat [up-sampled | encoder output l],
 *                       3x3 conv + ReLU (2 C_l -> C_l), 3x3 conv + ReLU;
 *   head:               1x1 conv (C0 -> cout), no activation.
 * All convolutions use zero padding and stride 1.  Max pooling routes the
 * gradient to the first maximum of each window in the order (0,0), (0,1),
 * (1,0), (1,1) (row, column).
 *
 * Flat FP32 parameter vector (ws_set_params / ws_get_params / ws_get_grads),
 * each layer's weights followed by its bias:
 *   for l = 0..L-1:   e1[l].W [C_l][3][3][cin_l]  e1[l].b [C_l]
 *                     e2[l].W [C_l][3][3][C_l]    e2[l].b [C_l]
 *                     (cin_0 = 8: the input is zero-padded to 8 channels;
 *                      cin_l = C_{l-1})
 *   for l = L-2..0:   up[l].W [2][2][C_l][C_{l+1}] ([dy][dx][out][in])
 *                     up[l].b [C_l]
 *                     d1[l].W [C_l][3][3][2 C_l] (input channels: up-sampled
 *                              first, then the skip)  d1[l].b [C_l]
 *                     d2[l].W [C_l][3][3][C_l]    d2[l].b [C_l]
 *   head.W [8][C0]  head.b [8]   (outputs cout..7 are padding)
 * Weight index order [out][ky][kx][in] means W[co][(ky*3+kx)*Cin + ci];
 * ky, kx = 0..2 address the input pixel (y + ky - 1, x + kx - 1).  The
 * transposed conv writes output pixel (2y+dy, 2x+dx) from input pixel (y, x).
 *
 * Numerics: activations are stored in BF16 (every layer output is rounded to
 * BF16 after bias and ReLU; the head output stays FP32); weights enter the
 * MFMA as BF16 copies of the FP32 masters; gradients of activations are
 * stored in BF16 (each is rounded once, where it is produced, and every
 * consumer takes it, times the ReLU mask, as a BF16 MFMA operand); products
 * accumulate in FP32; weight gradients are FP32; weight-gradient sums over pixels are
 * split in fixed chunks and reduced in a fixed order, so results are
 * deterministic.  The loss is accumulated in FP64.
 *
 * Conventions
 *   - Images are NHWC FP32 device arrays: x[b][y][x][c] with c fastest.
 *     ws_forward / ws_backward / ws_train_step take DEVICE pointers (use
 *     ws_malloc / ws_memcpy or any HIP allocation).  Parameter and gradient
 *     arrays passed to ws_set_params / ws_get_params / ws_get_grads are HOST
 *     arrays of exactly ws_num_params() floats.
 *   - All work is queued on the network's HIP stream (given at ws_create;
 *     NULL = the null stream), so it is ordered against other work there.
 *     The backward pass also runs its weight gradients on an internal stream
 *     of default priority that forks from and joins back into that stream
 *     (events), before the pass's last kernel.  Calls that return data to the
 *     host synchronise the network's stream; ws_destroy synchronises both.
 *   - Every call returns 0 (WS_OK) or a negative WS_E* code; the message of
 *     the last failure on the calling thread is ws_last_error().
 *   - The network owns its device buffers, sized for max_batch images.
 */
#ifndef WSNET_H
#define WSNET_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define WS_OK 0
#define WS_EINVAL (-1)  /* invalid argument or configuration */
#define WS_ENOMEM (-2)  /* device or host allocation failed  */
#define WS_EDEVICE (-3) /* a HIP runtime call failed          */

typedef struct ws_net ws_net; /* opaque, owned by the library */

typedef struct {
  int32_t levels;    /* L, 2..6                                               */
  int32_t base;      /* C0, multiple of 8                                     */
  int32_t cin;       /* input channels, 1..8                                  */
  int32_t cout;      /* output channels, 1..8                                 */
  int32_t H, W;      /* image size; divisible by 2^(L-1), and the lowest
                        level H W / 4^(L-1) a multiple of 64 pixels           */
  int32_t max_batch; /* largest batch passed to forward/backward             */
  int32_t conv_algo; /* 3x3 convolutions: 0 = direct kernels (an LDS-staged
                        8 x 32 pixel tile and its halo serve all nine taps)
                        at every level whose image is a whole number of such
                        tiles and whose channel counts are multiples of 32,
                        implicit GEMM elsewhere; 1 = implicit GEMM only.
                        Both give the same results up to FP32 summation
                        order.                                              */
} ws_config;

/* Allocates the network (parameters zero until ws_set_params). */
int ws_create(const ws_config *cfg, void *hip_stream, ws_net **out);
void ws_destroy(ws_net *net);

/* Number of FP32 parameters, and device bytes held by the network. */
int64_t ws_num_params(const ws_net *net);
int64_t ws_device_bytes(const ws_net *net);

/* Copies `count` (= ws_num_params) host floats into the parameters, resets
 * the Adam moments and step count and refreshes the BF16 weight copies. */
int ws_set_params(ws_net *net, const float *host, int64_t count);
int ws_get_params(ws_net *net, float *host, int64_t count);
/* Gradients of the last ws_backward (mean-squared-error loss). */
int ws_get_grads(ws_net *net, float *host, int64_t count);

/* y[batch][H][W][cout] = net(x[batch][H][W][cin]); device pointers;
 * asynchronous on the network's stream. */
int ws_forward(ws_net *net, const float *x, int32_t batch, float *y);

/* Forward on x, loss = mean over batch*H*W*cout of (y - target)^2, and the
 * gradient of that loss for every parameter (overwritten, not accumulated).
 * x, target: device [batch][H][W][cin|cout].  If loss is non-NULL the stream
 * is synchronised and the FP64 loss written to *loss. */
int ws_backward(ws_net *net, const float *x, const float *target, int32_t batch, double *loss);

/* One Adam step on the current gradients (bias-corrected moments; step count
 * kept by the network; weight_decay adds weight_decay * w to the gradient). */
int ws_adam(ws_net *net, float lr, float beta1, float beta2, float eps, float weight_decay);

/* ws_backward followed by ws_adam(lr, 0.9, 0.999, 1e-8, 0). */
int ws_train_step(ws_net *net, const float *x, const float *target, int32_t batch, float lr, double *loss);

/* Multiply-add FLOPs (2 per MAC) of one forward and one backward pass. */
int ws_flops(const ws_net *net, int32_t batch, double *fwd, double *bwd);

/* Device-memory helpers for callers without another HIP allocator.
 * kind: 0 host->device, 1 device->host, 2 device->device.  ws_memcpy first
 * waits for all work queued on the device, then copies synchronously. */
int ws_malloc(int64_t bytes, void **ptr);
int ws_free(void *ptr);
int ws_memcpy(void *dst, const void *src, int64_t bytes, int32_t kind);
int ws_sync(void);

const char *ws_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* WSNET_H */
