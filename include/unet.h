/*
 * unet.h -- C ABI of libunet.so: the 3-D U-Net that predicts a warm start for
 * the GMG Poisson solve (include/gmg.h), written for MI355X (gfx950).
 *
 * The network maps (sigma / s, L_x, L_y, L_z) to p / s on the same grid; GMG
 * then starts from that prediction, and the final GMG residual judges it
 * (plain GMG from zero remains the fallback).  It is not part of the paper's
 * method, which is the solver alone (Sec. 3); it is trained on solutions that
 * the solver itself produces.  Architecture (4 levels, channels 16-32-64-128):
 *   encoder level i: conv3x3x3 + ReLU, conv3x3x3 + ReLU, 2x2x2 average pool;
 *   decoder level i: nearest x2 upsample, conv3x3x3 + ReLU, concatenation with
 *   the encoder output of level i, two conv3x3x3 + ReLU;
 *   head: conv1x1x1 to one channel.  Zero padding, stride 1.
 *
 * Data layout (all DEVICE pointers):
 *   activations: BF16 (raw uint16 bits), channels-last [n][d][h][w][ld] with
 *   the tensor's channels at [off, off + C) of each voxel row of ld channels;
 *   ld, off and C multiples of 8 (16 for convolution outputs);
 *   weights: BF16 [C_out][taps][C_in] (taps = 27 in (kd, kh, kw) order, or 1);
 *   bias, gradients, master weights, Adam moments: FP32.
 *   A 3x3x3 convolution is the cross-correlation
 *     y[v][o] = b[o] + sum_{t, c} w[o][t][c] x[v + t - (1,1,1)][c]
 *   with zero padding; accumulation is FP32 (MFMA 16x16x32 BF16).
 *
 * Streams: every call enqueues on the given hipStream_t (NULL = legacy) and is
 * asynchronous except where a host scalar is returned.  Errors: UNET_EINVAL
 * for bad shapes or pointers (checked before any launch), UNET_EHIP for HIP
 * failures; unet_last_error() describes the last one.
 */
#ifndef UNET_H
#define UNET_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum unet_status { UNET_OK = 0, UNET_EINVAL = 1, UNET_ENOMEM = 3, UNET_EHIP = 4 } unet_status;

/* Activation view: base pointer, channels-last row length ld, channel offset
 * and count. */
typedef struct unet_act {
  void* p;
  int32_t ld, off, c;
} unet_act;

/* Grid of one activation: n samples of d x h x w voxels. */
typedef struct unet_shape {
  int32_t n, d, h, w;
} unet_shape;

/* y = act(conv(x, w) + bias).  taps = 27 (3x3x3) or 1 (1x1x1); relu 0/1.
 * out_f32: if non-NULL, FP32 output [voxels][y.ld] at channel y.off written
 * instead of the BF16 view y (y.p may then be NULL).  x.c multiple of 8 and
 * at most 256, y.c multiple of 16, fewer than 2^31 voxels (UNET_EINVAL
 * otherwise). */
unet_status unet_conv_fwd(unet_shape s, unet_act x, const void* w, const float* bias,
                          int32_t taps, unet_act y, float* out_f32, int32_t relu,
                          void* stream);

/* Which forward-convolution kernel unet_conv_fwd (and unet_conv_dgrad, a
 * forward convolution of dy) runs for these sizes (host only, no GPU call):
 * info[0] = 1 for LDS tiles (3x3x3 taps, 8, 16, 32 or 64 input channels,
 * 16-64 output channels, w a multiple of 64 and h of 4, or w = 32 and h a
 * multiple of 8), 0 for gathered operands (everything else); info[1] = tile
 * width (kind 1) or voxel blocks of 16 per wave (kind 0); info[2] = output
 * blocks of 16 per wave; info[3] = output-channel groups (workgroups that
 * share an input tile).  info: 4 int32 written by the call.  UNET_EINVAL for
 * a bad shape, channel count (cin a multiple of 8 up to 256; cout 16, 32, 64
 * or 128) or taps. */
unet_status unet_conv_kernel(unet_shape s, int32_t cin, int32_t cout, int32_t taps,
                             int32_t* info);

/* Data gradient of a convolution: dx = sum_{o, t} w[o][t][c] dy[v - t + 1][o]
 * (BF16 in, BF16 out; dx.c multiple of 16).  wflip: caller workspace of
 * C_out * taps * C_in BF16 for the flipped, transposed weights. */
unet_status unet_conv_dgrad(unet_shape s, unet_act dy, const void* w, int32_t taps,
                            unet_act dx, void* wflip, void* stream);

/* Weight and bias gradients: dw[o][t][c] = sum_v dy[v][o] x[v + t - 1][c],
 * db[o] = sum_v dy[v][o] (FP32 outputs, overwritten).  Deterministic split-K
 * over voxel chunks (FP32 partial rows summed in a fixed order): ws is caller
 * workspace of unet_wgrad_workspace() bytes (0 for invalid arguments).
 * Inputs: x.c = 8 or a multiple of 8, dy.c a multiple of 16, at most 128. */
size_t unet_wgrad_workspace(unet_shape s, int32_t cin, int32_t cout, int32_t taps);
unet_status unet_conv_wgrad(unet_shape s, unet_act x, unet_act dy, int32_t taps, float* dw,
                            float* db, void* ws, void* stream);

/* Which weight-gradient kernel unet_conv_wgrad runs for these sizes (host
 * only, no GPU call): info[0] = 1 for the row-tiled kernel (3x3x3 taps, w a
 * multiple of 32 or w = 16, h a multiple of 4, 8 or a multiple of 16 input
 * channels) else 0 for the voxel-chunk kernel; info[1..3] = input channels,
 * output channels and w extent of one row-kernel workgroup (0 otherwise);
 * info[4] = number of voxel chunks (partial rows); info[5] = d planes per
 * chunk (row kernel).  info: 6 int32 written by the call.  UNET_EINVAL for a
 * bad shape, channel count or taps. */
unet_status unet_wgrad_kernel(unet_shape s, int32_t cin, int32_t cout, int32_t taps,
                              int32_t* info);

/* dy_pre = dy * (y > 0) (ReLU backward, in place on dy allowed). */
unet_status unet_relu_bwd(unet_shape s, unet_act y, unet_act dy, unet_act out, void* stream);

/* 2x2x2 average pooling (s = fine shape, even d, h, w) and its gradient; nearest
 * x2 upsampling (s = coarse shape) and its gradient (sum over the 8 children).
 * Backward ops overwrite their output unless accumulate = 1 (then add). */
unet_status unet_pool_fwd(unet_shape fine, unet_act x, unet_act y, void* stream);
unet_status unet_pool_bwd(unet_shape fine, unet_act dy, unet_act dx, int32_t accumulate,
                          void* stream);
unet_status unet_up_fwd(unet_shape coarse, unet_act x, unet_act y, void* stream);
unet_status unet_up_bwd(unet_shape coarse, unet_act dy, unet_act dx, void* stream);

/* 1x1x1 head to one FP32 channel: y[v] = b + sum_c w[c] x[v][c] (w, b FP32).
 * Backward: dx[v][c] = w[c] dy[v] (skipped if dx.p is NULL), dw[c] = sum_v
 * dy[v] x[v][c], db = sum_v dy[v]; ws: unet_head_workspace() bytes. */
unet_status unet_head_fwd(unet_shape s, unet_act x, const float* w, const float* b, float* y,
                          void* stream);
size_t unet_head_workspace(unet_shape s, int32_t cin);
unet_status unet_head_bwd(unet_shape s, unet_act x, const float* w, const float* dy, unet_act dx,
                          float* dw, float* db, void* ws, void* stream);

/* Masked mean-squared error of an FP32 prediction [voxels] against target over
 * the cells with mask != 0: loss = sum (p - t)^2 / count.  Writes dpred =
 * 2 (p - t) mask / count (FP32), stats_dev[0..1] = (loss, count) on the
 * device (stats_dev: caller workspace of 2 + 512 doubles) and, if loss is not
 * NULL, the loss on the host (synchronises). */
unet_status unet_mse(unet_shape s, const float* pred, const float* target, const uint8_t* mask,
                     float* dpred, double* stats_dev, double* loss, void* stream);

/* Adam step on n FP32 master parameters with FP32 moments m, v, gradient g;
 * also writes the BF16 copy (may be NULL).  t = step number (1-based). */
unet_status unet_adam(int64_t n, float* master, float* m, float* v, const float* g,
                      void* bf16_out, float lr, float beta1, float beta2, float eps, int32_t t,
                      void* stream);

/* out[i] = a * in[i] (FP32; turns the network's p / s back into p). */
unet_status unet_scale(int64_t n, const float* in, float a, float* out, void* stream);

/* out[i] = a * (double)in[i] (FP64 out: the network's p / s as the initial
 * guess of the FP64 refinement solve). */
unet_status unet_scale_f64(int64_t n, const float* in, double a, double* out, void* stream);

/* FP32 -> BF16 (round to nearest even) and BF16 -> FP32 conversion. */
unet_status unet_to_bf16(int64_t n, const float* in, void* out, void* stream);
unet_status unet_from_bf16(int64_t n, const void* in, float* out, void* stream);

/* Network input: x[v][0..8) = (sigma/s, L_x, L_y, L_z, 0, 0, 0, 0) in BF16 from
 * FP32 fields [d][h][w] (sample k at offset k * d*h*w), with s given per
 * sample in `scale` (host array of n). */
unet_status unet_pack_input(unet_shape s, const float* sigma, const float* L,
                            const float* scale, void* x, void* stream);

/* Device self-check of the MFMA 16x16x32 BF16 operand/result lane layout the
 * convolutions assume: computes a 16x32 by 32x16 product with one MFMA and
 * writes it to out[16*16] (row-major) through that layout. */
unet_status unet_mfma_selfcheck(const void* a_bf16, const void* b_bf16, float* out, void* stream);

const char* unet_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* UNET_H */
