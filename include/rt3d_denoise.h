/*
 * rt3d_denoise.h -- C ABI of the learned heating-rate denoiser kernels.
 *
 * The paper's convergence study (sec. 2.4 and sec. 3.2, figure 2) shows the
 * Monte Carlo error falling as N_sample^-1/2 while the cost grows linearly
 * in N_sample.  This library adds a small 3D convolutional encoder-decoder
 * that maps low-photon heating tallies (plus the extinction field) to
 * high-photon ones; it is trained on tally pairs produced by the tracer
 * itself, and plain high-photon tracing remains the reference that measures
 * its error.  Not part of the paper's method.
 *
 * Conventions (all pointers are DEVICE pointers owned by the caller; every
 * call is asynchronous on `stream`, a hipStream_t passed as void*):
 *   activations  BF16 (uint16 bits) channels-last [D][H][W][C], C a multiple
 *                of 16 (or exactly 4 for the packed first layer, see
 *                rt3d_dn_conv3d_fwd);
 *   weights      BF16 [Cout][k^3][Cin] (k = 1 or 3), Cout a multiple of 32;
 *                FP32 master copies, gradients and Adam moments of the same
 *                shape; biases FP32 [Cout];
 *   convolution  stride 1, zero padding k/2, FP32 accumulation on the matrix
 *                cores (v_mfma_f32_32x32x16_bf16), BF16 output rounding to
 *                nearest even.
 * Errors: RT3D_EINVAL for bad arguments (checked before any launch),
 * RT3D_EDEVICE for a HIP failure (text in rt3d_dn_last_error()).
 */
#ifndef RT3D_DENOISE_H
#define RT3D_DENOISE_H

#include <stddef.h>
#include <stdint.h>

#include "rt3d.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Shape of one convolution: grid D x H x W, inputs c1 channels from x1 and
 * c2 (possibly 0) from x2, concatenated in that order; cout outputs.  With
 * up1 != 0 (ksize 3, D, H, W even) x1 is stored at half resolution
 * [D/2][H/2][W/2][c1] and read nearest-upsampled: voxel (z, y, x) of the
 * input is x1[z/2][y/2][x/2] (the decoder's upsampling, never written out). */
typedef struct {
    int32_t D, H, W;
    int32_t c1, c2, cout;
    int32_t ksize; /* 1 or 3 */
    int32_t up1;
    int32_t yf_cols; /* FP32 output keeps channels [0, yf_cols) only, with
                        row stride yf_cols; 0 = cout */
} rt3d_dn_conv;

const char* rt3d_dn_last_error(void);

/* y = act(conv(concat(x1, x2), w) + bias); act = ReLU if relu != 0.
 * c1 is a multiple of 16, or exactly 4 for a 3x3x3 convolution to 32
 * outputs with no second input, no upsampling and o1 = 32 (the first layer:
 * x1 [vox][4], w [32][27][4]; three x-taps share one MFMA K-chunk).
 * Output channels [0, o1) go to y1 ([vox][o1]), [o1, cout) to y2
 * ([vox][cout - o1], o1 a multiple of 32).  If yf is not NULL the FP32
 * values of channels [0, yf_cols) are also written to yf [vox][yf_cols] (y1
 * may then be NULL when o1 == cout).  bias may be NULL.  With flipped weights (rt3d_dn_flip_weights)
 * and no bias/activation this computes the data gradient. */
rt3d_status rt3d_dn_conv3d_fwd(const rt3d_dn_conv* c, const uint16_t* x1, const uint16_t* x2, const uint16_t* w,
                               const float* bias, int32_t relu, uint16_t* y1, uint16_t* y2, int32_t o1, float* yf,
                               void* stream);

/* The network's last two layers in one launch (inference): a 3x3x3
 * convolution to exactly 32 channels, y = act(conv(concat(x1, x2), w) +
 * bias) rounded to BF16 (c1, c2 multiples of 16; up1 as above), followed by
 * the 1x1x1 head hw [32][32] (output channel, input channel) with bias hb
 * (may be NULL).  Only the FP32 head channels [0, hcols) are written, to
 * hy [vox][hcols] (1 <= hcols <= 32); y itself is never stored.  The result
 * is bitwise that of rt3d_dn_conv3d_fwd for the convolution followed by
 * rt3d_dn_conv3d_fwd for the head (same products in the same order).
 * RT3D_EINVAL on a NULL required pointer or an unsupported shape. */
rt3d_status rt3d_dn_conv3d_fwd_head(const rt3d_dn_conv* c, const uint16_t* x1, const uint16_t* x2, const uint16_t* w,
                                    const float* bias, int32_t relu, const uint16_t* hw, const float* hb, int32_t hcols,
                                    float* hy, void* stream);

/* The first layer followed by the 2x2x2 average pooling of its output, in
 * one launch (inference): c describes the packed first layer (c1 = 4, c2 =
 * 0, ksize 3, cout 32, up1 0, yf_cols 0) on even D, H, W.  y receives the
 * BF16 layer output [D][H][W][32] and ypool its pooling [D/2][H/2][W/2][32],
 * both bitwise equal to rt3d_dn_conv3d_fwd (y1 = y, o1 = 32) followed by
 * rt3d_dn_pool2; the full-resolution output is not read back.  c1 = 5: the
 * network with the direct-beam input, x1 BF16 [D][H][W][8] (channels 5-7
 * zero) and w the 16-channel weights [32][27][16] (channels 0-4 used); one
 * MFMA K-chunk holds the 15 products of three x-taps, so the output equals
 * rt3d_dn_conv3d_fwd on 16-channel features up to the order of the
 * products within a chunk.  Device pointers; RT3D_EINVAL for any other
 * shape. */
rt3d_status rt3d_dn_conv3d_fwd_pool(const rt3d_dn_conv* c, const uint16_t* x1, const uint16_t* w, const float* bias,
                                    int32_t relu, uint16_t* y, uint16_t* ypool, void* stream);

/* wt[ci][k^3 - 1 - t][co] = w[co][t][ci]: the kernel of the data gradient. */
rt3d_status rt3d_dn_flip_weights(const uint16_t* w, uint16_t* wt, int32_t cout, int32_t cin, int32_t ksize,
                                 void* stream);

/* dw[co][t][ci] += sum_v dz[v][co] x[v + offset(t)][ci] (FP32, accumulated
 * with atomics: clear dw first); db[co] += sum_v dz[v][co] if db != NULL.
 * x = concat(x1, x2) is the forward input (c->up1 must be 0), dz the
 * gradient at the convolution output (after the activation's derivative). */
rt3d_status rt3d_dn_conv3d_wgrad(const rt3d_dn_conv* c, const uint16_t* x1, const uint16_t* x2, const uint16_t* dz,
                                 float* dw, float* db, void* stream);

/* Bytes of workspace rt3d_dn_conv3d_wgrad_ws needs for this shape (0 on bad
 * arguments).  Host call. */
size_t rt3d_dn_wgrad_workspace_size(const rt3d_dn_conv* c);

/* rt3d_dn_conv3d_wgrad with a caller-owned DEVICE workspace (at least
 * rt3d_dn_wgrad_workspace_size bytes, 256-byte aligned, contents need not be
 * initialised): every row chunk of the reduction stores its partial dw (and
 * every block its partial db) there, and the partials are added to dw / db
 * in a fixed order, so the result does not depend on scheduling (bitwise
 * reproducible; the plain variant adds with FP32 atomics). */
rt3d_status rt3d_dn_conv3d_wgrad_ws(const rt3d_dn_conv* c, const uint16_t* x1, const uint16_t* x2,
                                    const uint16_t* dz, float* dw, float* db, void* workspace,
                                    size_t workspace_bytes, void* stream);

/* dz = dy where y > 0 else 0 (ReLU derivative through its output y). */
rt3d_status rt3d_dn_relu_bwd(const uint16_t* dy, const uint16_t* y, uint16_t* dz, uint64_t n, void* stream);

/* out = a + b elementwise (BF16). */
rt3d_status rt3d_dn_add(const uint16_t* a, const uint16_t* b, uint16_t* out, uint64_t n, void* stream);

/* 2x2x2 average pooling of x [D][H][W][C] into y [D/2][H/2][W/2][C] (C a
 * multiple of 8 and x, y 16-byte aligned; each output is the BF16 rounding
 * of 1/8 of the FP32 sum of its 8 inputs taken in z, y, x order); with
 * backward != 0, x is the gradient at the pooled output and y receives the
 * gradient at the input (each input voxel gets 1/8 of its parent's). */
rt3d_status rt3d_dn_pool2(const uint16_t* x, uint16_t* y, int32_t D, int32_t H, int32_t W, int32_t C,
                          int32_t backward, void* stream);

/* Nearest-neighbour 2x upsampling of x [D][H][W][C] into y [2D][2H][2W][C];
 * with backward != 0, x is the gradient at the upsampled output
 * ([2D][2H][2W][C]) and y [D][H][W][C] receives the sum over children. */
rt3d_status rt3d_dn_up2(const uint16_t* x, uint16_t* y, int32_t D, int32_t H, int32_t W, int32_t C,
                        int32_t backward, void* stream);

/* Residual head and squared-error loss: pred[v][c] = out[v][c] + base[v][c]
 * for c < nout (out is FP32 [vox][cpad], base/target/pred FP32 [vox][nout]);
 * if target != NULL: *loss += sum (pred - target)^2 (FP64) and dout[v][c] =
 * 2 (pred - target) / (nvox nout) (BF16 [vox][cpad], 0 in padding).  pred,
 * dout, loss may be NULL. */
rt3d_status rt3d_dn_mse(const float* out, int32_t cpad, const float* base, const float* target, int32_t nout,
                        uint64_t nvox, float* pred, uint16_t* dout, double* loss, void* stream);

/* One Adam step (Kingma and Ba) on n FP32 parameters p with gradient g and
 * moments m1, m2; step counts from 1; pb (may be NULL) receives BF16 p. */
rt3d_status rt3d_dn_adam(float* p, const float* g, float* m1, float* m2, uint16_t* pb, uint64_t n, float lr,
                         float b1, float b2, float eps, int32_t step, void* stream);

/* y = BF16(x). */
rt3d_status rt3d_dn_to_bf16(const float* x, uint16_t* y, uint64_t n, void* stream);

/* Network input per voxel: channel 0 = hdir/scale, 1 = hdif/scale,
 * 2 = ln(1 + 20 k_ext dz), 3 = ln(1 + 200 k_abs dz), with direct != NULL
 * channel 4 = direct/scale (FP32 [vox], cpad >= 5), the rest 0
 * (feat BF16 [vox][cpad], cpad 4, 8 or a multiple of 16); base FP32 [vox][2] = (hdir/scale, hdif/scale), the
 * residual the network corrects (NULL: not written).  hdir, hdif: FP32 heating fields; k_ext,
 * k_abs: FP32 [vox] extinction and absorption coefficients (m^-1). */
rt3d_status rt3d_dn_features(const float* hdir, const float* hdif, const float* k_ext, const float* k_abs, float dz,
                             float scale, uint64_t nvox, int32_t cpad, const float* direct, uint16_t* feat, float* base,
                             void* stream);

/* Direct-beam feature (an optional fifth network input, channel 4 of
 * rt3d_dn_features = direct/scale): a deterministic estimate of the heating
 * by the unscattered sun beam, in a gray medium k_ext, k_abs (FP32 device
 * [nz][ny][nx], e.g. flux-weighted over g-points).  The beam's transmittance
 * at every cell centre is carried down level by level (read bilinearly,
 * periodic in x and y, from the level above where the sun ray through the
 * centre meets it; half the path in each level); a cell absorbs
 * T_entry (1 - exp(-k_ext dz / mu0)) k_abs / k_ext of the direct flux
 * (T_entry: half a level above the centre), times direct_fraction and
 * layer_scale[k] (FP64 device [nz], e.g. the heating-rate conversion).
 * out: FP32 device [nz][ny][nx]; work: FP32 device [2][ny][nx].  A feature
 * for the network, not the method's estimate (no scattering, no surface). */
typedef struct {
    int32_t nx, ny, nz;
    float dx, dy, dz;
    float sun_x, sun_y, sun_z;  /* propagation direction of the beam (unit, sun_z < 0) */
    float direct_fraction;
} rt3d_dn_direct;
rt3d_status rt3d_dn_direct_feature(const rt3d_dn_direct* d, const float* k_ext, const float* k_abs,
                                   const double* layer_scale, float* out, float* work, void* stream);

/* Field scale of the network input: work[0] = (mean hdir + mean hdif) / 2
 * (1 if that is not positive), summed in FP64 in a fixed order (bitwise
 * reproducible).  hdir, hdif: FP32 device [nvox]; work: FP64 device
 * [RT3D_DN_SCALE_WORK] (work[1..] are partial sums). */
#define RT3D_DN_SCALE_WORK 2049
rt3d_status rt3d_dn_field_scale(const float* hdir, const float* hdif, uint64_t nvox, double* work, void* stream);

/* Inference output in one pass: hdir[v] = max(out[v][0] + base0, 0) scale,
 * hdif[v] = max(out[v][1] + base1, 0) scale with (base0, base1) the residual
 * base rt3d_dn_features forms from hdir_in, hdif_in and scale; bitwise
 * rt3d_dn_features' base, rt3d_dn_mse (pred) and rt3d_dn_unfeature in turn.
 * out: FP32 [nvox][cpad] network output; all FP32 device arrays. */
rt3d_status rt3d_dn_residual_unfeature(const float* out, int32_t cpad, const float* hdir_in, const float* hdif_in,
                                       float scale, uint64_t nvox, float* hdir, float* hdif, void* stream);

/* hdir[v] = max(pred[v][0], 0) scale, hdif[v] = max(pred[v][1], 0) scale. */
rt3d_status rt3d_dn_unfeature(const float* pred, float scale, uint64_t nvox, float* hdir, float* hdif,
                              void* stream);

#ifdef __cplusplus
}
#endif

#endif /* RT3D_DENOISE_H */
