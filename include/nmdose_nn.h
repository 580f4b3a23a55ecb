/*
 * nmdose_nn.h -- C ABI of the learned denoiser of the dosimetry engine.
 *
 * Not part of the paper: this is the learned stage added on top of the Monte
 * Carlo of Section 2.  A 3D U-Net maps a low-history dose map plus density
 * and activity to the high-history dose map; the Monte Carlo of nmdose.h
 * generates its training data and stays its fallback and judge.  The calls
 * below are the network's kernels: the Python driver owns the tensors and
 * sequences the calls, and performs no arithmetic of its own.
 *
 * Conventions (in addition to those of nmdose.h)
 *   Activations are bfloat16 (stored as uint16_t bit patterns), channels
 *   last: [n][d][h][w][c], c fastest.  Channel counts are multiples of 8 and
 *   every tensor pointer is 16-byte aligned.  d, h, w play the roles of z, y,
 *   x of the dose map.
 *   A 3x3x3 convolution weight is bfloat16 [c_out][27][c_in] with tap
 *   t = (kz*3 + ky)*3 + kx applied to the input voxel (z+kz-1, y+ky-1,
 *   x+kx-1); voxels outside the volume read as zero (padding 1).  Its
 *   "flipped" copy is [c_in][27][c_out] with w_t[i][t][o] = w[o][26-t][i];
 *   the backward-data pass reads it.
 *   Products accumulate in FP32 (BF16 x BF16 matrix-core instructions);
 *   results stored as bfloat16 are rounded to nearest, ties to even.
 *   Every call is asynchronous on the context stream and returns a status;
 *   all pointers are device pointers unless documented as host.
 */
#ifndef NMDOSE_NN_H
#define NMDOSE_NN_H

#include <stdint.h>

#include "nmdose.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Input of a convolution: the channel concatenation [x0 | x1].  The first
 * c0 channels come from x0 -- at full resolution, or, if up0 != 0, from a
 * tensor of half resolution ((d+1)/2, (h+1)/2, (w+1)/2) up-sampled by two
 * with nearest-neighbour (voxel (z, y, x) reads (z/2, y/2, x/2)).  The next
 * c1 channels come from x1 at full resolution (x1 = NULL and c1 = 0 when
 * there is no second part). */
typedef struct {
  const uint16_t *x0;
  int32_t c0;
  int32_t up0;
  const uint16_t *x1;
  int32_t c1;
} nmd_nn_src;

/* y = epilogue(conv3x3(x, weight) + bias): bias (FP32 [c_out], or NULL) is
 * added, then ReLU if relu != 0, then, if mask is given ([n][d][h][w][c_out]
 * bfloat16), every element whose mask element is not > 0 is set to zero.
 * c_in = x->c0 + x->c1 must be 8, 16, 32, 48, 64 or 96 and c_out 16, 32, 48,
 * 64 or 96 (the layer shapes of the network and of its backward pass). */
nmd_status nmd_conv3d_fwd(nmd_ctx *ctx, int32_t n, int32_t d, int32_t h, int32_t w,
                          const nmd_nn_src *x, const uint16_t *weight, const float *bias,
                          int32_t c_out, int32_t relu, const uint16_t *mask, uint16_t *y);

/* Gradient with respect to the input of y = conv3x3(x, w): dx = the
 * zero-padded correlation of dy with the flipped weight w_t, then, if mask
 * is given ([..][c_in]), zeroed where the mask is not > 0 (the ReLU of the
 * layer that produced x).  dy has c_out channels, dx c_in. */
nmd_status nmd_conv3d_bwd_data(nmd_ctx *ctx, int32_t n, int32_t d, int32_t h, int32_t w,
                               const uint16_t *dy, int32_t c_out, const uint16_t *weight_t,
                               int32_t c_in, const uint16_t *mask, uint16_t *dx);

/* Gradient with respect to the weight and bias of y = conv3x3(x, w) + b:
 * dw[o][t][i] = sum over voxels of dy[v][o] x[v + offset(t)][i] and
 * db[o] = sum over voxels of dy[v][o], both FP32 (db may be NULL).  The sums
 * run over fixed per-workgroup partials in a fixed order, so the result is
 * reproducible bit for bit.  Uses a context-owned workspace (allocated on
 * first use, grown when needed). */
nmd_status nmd_conv3d_bwd_weight(nmd_ctx *ctx, int32_t n, int32_t d, int32_t h, int32_t w,
                                 const nmd_nn_src *x, const uint16_t *dy, int32_t c_out,
                                 float *dw, float *db);

/* 2x2x2 average pool: y[n][z][y][x][c] = mean of the 8 voxels of x at
 * (2z+a, 2y+b, 2x+e); d, h, w are the dimensions of x (all even). */
nmd_status nmd_nn_pool2(nmd_ctx *ctx, int32_t n, int32_t d, int32_t h, int32_t w, int32_t c,
                        const uint16_t *x, uint16_t *y);

/* Backward helper at one level of the network:
 *   out[v][i] = [mask[v][i] > 0] * (a[v*a_stride + a_off + i] + B(v, i))
 * with, by b_mode:
 *   0  B = 0;
 *   1  B = sum of b over the 8 voxels of the level above (dimensions
 *      2d x 2h x 2w) whose nearest-neighbour parent is v: the backward of
 *      the x2 up-sample; b has b_stride channels, read from b_off;
 *   2  B = b[parent of v] / 8 from the level below (dimensions d/2 x h/2 x
 *      w/2, d, h, w even): the backward of the 2x2x2 average pool.
 * a may be NULL (no term); mask may be NULL (no masking).  out has c
 * channels; strides and offsets are multiples of 8. */
nmd_status nmd_nn_combine(nmd_ctx *ctx, int32_t n, int32_t d, int32_t h, int32_t w, int32_t c,
                          const uint16_t *mask, const uint16_t *a, int32_t a_stride,
                          int32_t a_off, int32_t b_mode, const uint16_t *b, int32_t b_stride,
                          int32_t b_off, uint16_t *out);

/* Network input for the box box[6] = {z0, y0, x0, d, h, w} of a phantom of
 * dimensions nz x ny x nx (maps [nz][ny][nx]):
 *   scale[0] = mean of dose_lo over body voxels (label > 0) of the box,
 *   scale[1] = mean of activity over the same voxels (1 where the mean is 0),
 *   x0[v] = bf16(dose_lo/scale[0], density/1.85, activity/scale[1], 0 x 5),
 *   target[v] = (float)(dose_hi/scale[0]) if target and dose_hi are given.
 * dose_lo, dose_hi: FP64; density, activity: FP32; label: uint8; x0 has 8
 * channels; scale is a device double[2]. */
nmd_status nmd_nn_prepare(nmd_ctx *ctx, int32_t nz, int32_t ny, int32_t nx, const int32_t *box,
                          const double *dose_lo, const double *dose_hi, const float *density,
                          const float *activity, const uint8_t *label, uint16_t *x0,
                          float *target, double *scale);

/* Head, loss and the head's backward for one batch of nvox voxels:
 *   pred[v] = x0[v][0] + sum_i head_w[i] feat[v][i] + head_b[0]   (FP32)
 *   w[v]    = 1 / max(target[v], weight_floor) if weight_floor > 0, else 1
 *   loss    = sum_v w[v] (pred[v] - target[v])^2
 *   g[v]    = 2 w[v] (pred[v] - target[v]) / nvox
 *   dfeat[v][i] = [feat[v][i] > 0] * bf16(g[v] head_w[i])
 *   grad[0..15] = sum_v g[v] feat[v][i],  grad[16] = sum_v g[v],
 *   grad[17] = loss.
 * The weight is the inverse of the target, a variance proxy: Monte Carlo
 * dose noise has a variance roughly proportional to the dose.  feat has 16
 * channels, x0 8; head_w FP32[16], head_b FP32[1]; grad is a device
 * float[18]. */
nmd_status nmd_nn_head_loss(nmd_ctx *ctx, int64_t nvox, const uint16_t *feat,
                            const uint16_t *x0, const float *target, const float *head_w,
                            const float *head_b, float weight_floor, uint16_t *dfeat,
                            float *grad);

/* Head at inference: for every voxel v of the box (box as nmd_nn_prepare),
 * out[full-map voxel] = max(pred[v], 0) * scale[0] (FP64); voxels of out
 * outside the box are not written. */
nmd_status nmd_nn_head_infer(nmd_ctx *ctx, int32_t nz, int32_t ny, int32_t nx,
                             const int32_t *box, const uint16_t *feat, const uint16_t *x0,
                             const float *head_w, const float *head_b, const double *scale,
                             double *out);

/* One Adam step (Kingma and Ba 2015, Algorithm 1, bias-corrected) on n FP32
 * parameters theta with moments m, v and gradient grad; step counts from
 * 1.  If w_bf16 is given, writes the bfloat16 working copy of theta
 * (theta viewed as [c_out][27][c_in]); if w_t_bf16 is given, also its
 * flipped copy (layout above).  c_out, c_in are ignored when both are NULL. */
nmd_status nmd_nn_adam(nmd_ctx *ctx, float *theta, float *m, float *v, const float *grad,
                       int64_t n, int32_t step, float lr, float beta1, float beta2, float eps,
                       uint16_t *w_bf16, uint16_t *w_t_bf16, int32_t c_out, int32_t c_in);

/* The bfloat16 working copy and flipped copy of an FP32 weight [c_out][27][c_in]
 * (either output may be NULL). */
nmd_status nmd_nn_cast_weight(nmd_ctx *ctx, const float *theta, int32_t c_out, int32_t c_in,
                              uint16_t *w_bf16, uint16_t *w_t_bf16);

/* Organ means (Eq. 2 of Section 2.4) of a caller-supplied per-voxel map of
 * the registered phantom phantom_id (device FP64 [nz][ny][nx], for example a
 * denoised dose-rate map): out[o-1] = mean of map over the voxels with label
 * o, o = 1..n_organs (host FP64).  Synchronises the stream. */
nmd_status nmd_organ_mean_map(nmd_ctx *ctx, int32_t phantom_id, const double *map,
                              int32_t n_organs, double *out);

/* nmd_organ_mean_map for callers that cannot allocate (code under HIP graph
 * capture, allocation-free serving loops, harnesses that forbid hipMalloc):
 * same arguments, results and errors, but the call makes no device
 * allocation (no hipMalloc or hipFree) and, when it succeeds, no host heap
 * allocation either.  Its per-label partial sums live in a library-owned
 * static device buffer of 256 FP64 slots (2 KiB per device, kept until the
 * process ends), cleared by a fill kernel at the start of every call; a
 * phantom with more than 255 labels is refused with NMD_E_UNSUPPORTED (labels
 * are 8-bit, so none can have more).  Every call on a device shares that
 * device's buffer: calls that overlap on one device (from several threads or
 * contexts on different streams) race and must be serialised by the caller.
 * Synchronises the stream. */
nmd_status nmd_organ_mean_map_noalloc(nmd_ctx *ctx, int32_t phantom_id, const double *map,
                                      int32_t n_organs, double *out);

/* Test hook: one 16x16x32 BF16 matrix-core product, d = a * b with a
 * row-major bfloat16 [16][32], b row-major [32][16], d row-major FP32 [16][16]. */
nmd_status nmd_debug_mfma(nmd_ctx *ctx, const uint16_t *a, const uint16_t *b, float *d);

#ifdef __cplusplus
}
#endif

#endif /* NMDOSE_NN_H */
