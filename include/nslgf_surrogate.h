/*
 * nslgf_surrogate.h -- C ABI of the learned surrogate's kernels (BF16 MFMA, FP32 accumulation).
 *
 * The surrogate is a 3D convolutional U-Net that proposes the vorticity several IF-HERK steps ahead;
 * the plain step of nslgf.h judges every proposal and replaces it when it is off (the surrogate is
 * not part of the paper).  These entry points are its layers, forward and backward, so that training
 * and inference run entirely in the library's kernels; network wiring lives in the caller.
 *
 * Conventions: volumes are D*H*W voxels (x fastest) stored channels-last, [voxel][channel];
 * activations for the matrix cores are BF16 (uint16 storage, round-to-nearest-even), everything
 * else FP32.  Convolutions are 3x3x3, stride 1, zero padding 1, no bias.  Weights are
 * [27 taps][Cout][Cin], tap = (dz+1)*9 + (dy+1)*3 + (dx+1).  All pointers are device pointers of the
 * handle's device; calls are asynchronous on `stream`; errors as in nslgf.h.
 * Shape rules: Cin % 16 == 0, Cout % 32 == 0, D*H*W % 32 == 0 (violations give NSLGF_EINVAL).
 */
#ifndef NSLGF_SURROGATE_H
#define NSLGF_SURROGATE_H

#include "nslgf.h"

#ifdef __cplusplus
extern "C" {
#endif

/* y[v][co] = act(sum_{tap,ci} x[v + off(tap)][ci] w[tap][co][ci]), act = ReLU if relu, FP32 y. */
int sur_conv3d_fwd(nslgf_t h, const void *x_bf16, const void *w_bf16, void *y_f32, int D, int H, int W, int cin,
                   int cout, int relu, void *stream);
/* dx[v][ci] = sum_{tap,co} dy[v - off(tap)][co] w[tap][co][ci] (FP32 dx); wt_bf16 is the transposed
 * weight [27][cin][cout] from sur_weight_transpose. */
int sur_conv3d_bwd_data(nslgf_t h, const void *dy_bf16, const void *wt_bf16, void *dx_f32, int D, int H, int W,
                        int cin, int cout, void *stream);
/* dw[tap][co][ci] = sum_v dy[v][co] x[v + off(tap)][ci] (FP32, overwritten), deterministic split
 * over voxel chunks with a fixed-order reduction; `work` must hold sur_bwd_weight_work_bytes(). */
int sur_conv3d_bwd_weight(nslgf_t h, const void *dy_bf16, const void *x_bf16, void *dw_f32, void *work, int D, int H,
                          int W, int cin, int cout, void *stream);
size_t sur_bwd_weight_work_bytes(int D, int H, int W, int cin, int cout);
/* wt[tap][ci][co] = w[tap][co][ci] (BF16) */
int sur_weight_transpose(nslgf_t h, const void *w_bf16, void *wt_bf16, int cin, int cout, void *stream);

/* Elementwise / resampling layers on channels-last FP32 tensors (n = voxels * channels): */
int sur_cast_bf16(nslgf_t h, const void *x_f32, void *y_bf16, long long n, void *stream);
int sur_relu_bwd(nslgf_t h, const void *y_f32, void *g_f32, long long n, void *stream); /* g *= (y > 0) */
int sur_add(nslgf_t h, const void *a_f32, const void *b_f32, void *out_f32, long long n, void *stream);
/* 2x2x2 average pooling (D, H, W even) and its adjoint; nearest 2x upsampling and its adjoint.
 * D, H, W are the FINE sizes in all four calls. */
int sur_pool2_fwd(nslgf_t h, const void *x, void *y, int D, int H, int W, int c, void *stream);
int sur_pool2_bwd(nslgf_t h, const void *gy, void *gx, int D, int H, int W, int c, void *stream);
int sur_up2_fwd(nslgf_t h, const void *x, void *y, int D, int H, int W, int c, void *stream);
int sur_up2_bwd(nslgf_t h, const void *gy, void *gx, int D, int H, int W, int c, void *stream);
/* Squared error over the first `used` of `c` channels: grad[v][k] = 2 (pred - target) / (nvox used)
 * for k < used, 0 otherwise; per-block partial sums of the squared error go to partial_f64
 * (`nblocks` of them, nblocks = 1024); the caller sums them. target is [voxel][used] FP32. */
int sur_mse(nslgf_t h, const void *pred, const void *target, void *grad, void *partial_f64, long long nvox, int c,
            int used, void *stream);
/* sur_mse with the gradient written only as its BF16 copy y_bf16 [voxel][c] and, when yb_bf16 is given, its
 * blocked copy (the layout of sur_to_blocked8): the same bits as sur_mse followed by sur_cast_bf16_ex of
 * the gradient, without the FP32 gradient; partial_f64 as sur_mse (1024 per-block sums, summed in another
 * fixed order).  nvox % 8 == 0, c % 8 == 0, y_bf16 and yb_bf16 16-byte aligned. */
int sur_mse_cast(nslgf_t h, const void *pred, const void *target, void *partial_f64, void *y_bf16, void *yb_bf16,
                 long long nvox, int c, int used, void *stream);
/* Adam step on FP32 master weights (t = step number from 1) and their BF16 copy. */
int sur_adam(nslgf_t h, void *w, void *w_bf16, const void *g, void *m, void *v, long long n, float lr, float b1,
             float b2, float eps, int t, void *stream);
/* The convolution, layout and fused-cast calls move 16 bytes per access: their tensors must start on
 * 16-byte boundaries (NSLGF_EINVAL otherwise). */
/* Blocked BF16 layout of the weight gradient's operands: [nvox / 8][c][8] (8 consecutive voxels of one
 * channel contiguous).  sur_to_blocked8 rearranges a channels-last [nvox][c] BF16 tensor into it
 * (nvox % 8 == 0, c % 8 == 0, xb must not overlap x). */
int sur_to_blocked8(nslgf_t h, const void *x_bf16, void *xb_bf16, long long nvox, int c, void *stream);
/* Cast of a channels-last FP32 tensor [nvox][c] to BF16 with an optional ReLU backward (act_f32: the
 * layer's activation; values where act is not > 0 become +0, as sur_relu_bwd leaves them) and an
 * optional blocked copy (yb_bf16, may be NULL): y = bf16(val) channels-last, yb the same values in the
 * blocked layout.  Equal bit for bit to sur_relu_bwd, sur_cast_bf16 and sur_to_blocked8 in turn, without
 * writing the FP32 tensor back.  nvox % 8 == 0, c % 8 == 0. */
int sur_cast_bf16_ex(nslgf_t h, const void *src_f32, const void *act_f32, void *y_bf16, void *yb_bf16,
                     long long nvox, int c, void *stream);
/* Resampling, skip sum and cast in one pass: val[v][ch] = scale * coarse[parent(v)][ch] + skip[v][ch] over the
 * fine grid [D][H][W] (channels-last, c channels), parent(v) = (z/2, y/2, x/2) in the coarse grid
 * [D/2][H/2][W/2]; then as sur_cast_bf16_ex (ReLU backward of act when act is given, BF16 copy y, blocked
 * copy yb when yb is given).  scale 1 gives sur_up2_fwd, sur_add and sur_cast_bf16_ex in turn, scale 1/8
 * sur_pool2_bwd, sur_add and sur_cast_bf16_ex, bit for bit, without writing the two FP32 tensors.  Even
 * D, H, W with D*H*W % 8 == 0, c % 8 == 0, 16-byte aligned tensors (else NSLGF_EINVAL). */
int sur_cast_bf16_up(nslgf_t h, const void *coarse_f32, double scale, const void *skip_f32, const void *act_f32,
                     void *y_bf16, void *yb_bf16, int D, int H, int W, int c, void *stream);
/* Weight gradient from operands already in the blocked layout (dyb [nvox/8][cout][8], xb [nvox/8][cin][8]):
 * the result of sur_conv3d_bwd_weight bit for bit, without its two layout copies.  Needs W % 8 == 0 and
 * D*H*W % 16 == 0 (else NSLGF_EINVAL); work of sur_bwd_weight_blocked_work_bytes bytes. */
int sur_conv3d_bwd_weight_blocked(nslgf_t h, const void *dyb_bf16, const void *xb_bf16, void *dw_f32, void *work,
                                  int D, int H, int W, int cin, int cout, void *stream);
size_t sur_bwd_weight_blocked_work_bytes(int D, int H, int W, int cin, int cout);
/* Pack planar FP64 vorticity [3][D][H][W] into the network input [voxel][16] BF16:
 * channels 0..2 = omega * scale, channel 3 = feat, the rest 0. */
int sur_pack_input(nslgf_t h, const void *omega_f64, void *x_bf16, int D, int H, int W, double scale, double feat,
                   void *stream);
/* Input of the correction form, whose network refines the linear extrapolation of one plain step:
 * channels 0..2 = omega * scale, channel 3 = feat, channels 4..6 = delta * dscale (delta: planar FP64
 * [3][D][H][W], the change of the vorticity over one plain step), the rest 0. */
int sur_pack_input_pair(nslgf_t h, const void *omega_f64, const void *delta_f64, void *x_bf16, int D, int H, int W,
                        double scale, double dscale, double feat, void *stream);
/* out[i] = ca a[i] + cb b[i] + cc c[i] for i < n (FP64; c may be NULL, then the last term is left out).
 * Forms the extrapolation w_k + h (w_{k+1} - w_k), the one-step change and the correction targets. */
int sur_combine3(nslgf_t h, const void *a_f64, const void *b_f64, const void *c_f64, void *out_f64, long long n,
                 double ca, double cb, double cc, void *stream);
/* Pack a planar FP64 target field [3][D][H][W] times scale into [voxel][3] FP32. */
int sur_pack_target(nslgf_t h, const void *f_f64, void *t_f32, int D, int H, int W, double scale, void *stream);
/* Unpack: out[q][v] = base[q][v] + y[v][q] / scale for q < 3 (planar FP64). */
int sur_unpack_update(nslgf_t h, const void *base_f64, const void *y_f32, void *out_f64, int D, int H, int W, int c,
                      double scale, void *stream);
/* Self-check of the matrix-core operand layout: one v_mfma_f32_32x32x16_bf16 on a 32x16 A and a
 * 16x32 B given row-major (BF16), writing the 32x32 FP32 product row-major. */
int sur_mfma_selftest(nslgf_t h, const void *a_bf16, const void *b_bf16, void *c_f32, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* NSLGF_SURROGATE_H */
