/* lbm_nn.h -- C ABI of the kernels behind the learned warm start of the
 * solver: a 3D convolutional encoder-decoder (the surrogate) that maps a
 * solid mask and a component-fraction field to near-steady velocity and
 * component densities, which the solver then takes as its initial state
 * through lbm_set_fields (lbm.h) and runs to convergence, so the method
 * itself is never changed.  The paper has no such component: it is an
 * accelerator around the method, whose output the solver always judges.
 *
 * Conventions shared by every call:
 *   - all tensor pointers are device pointers, owned by the caller; no call
 *     allocates, frees or keeps a pointer after it returns;
 *   - activations are channel-last: element (p, c) of a view (ptr, ld) is
 *     ptr[p * ld + c] for positions p = ((b * D + z) * H + y) * W + x;
 *     a view may start inside a wider tensor (a channel offset), which is
 *     how channel concatenation costs nothing;
 *   - "bf16" tensors hold bfloat16 bit patterns (uint16_t), rounded to
 *     nearest even; arithmetic accumulates in FP32;
 *   - the convolution is 3 x 3 x 3 with periodic padding (the lattices are
 *     periodic); weights w[t][co][ci] with tap t = 9 (dz + 1) + 3 (dy + 1)
 *     + (dx + 1):  y[p][co] = b[co] + sum_t sum_ci w[t][co][ci] x[p + d_t][ci];
 *   - stream is a hipStream_t (NULL = the default stream); calls only
 *     enqueue work;
 *   - return 0 on success, LBM_EINVAL (lbm.h) for unsupported sizes or
 *     misaligned views (checked on the host before anything is enqueued),
 *     LBM_EDEVICE if the launch fails.
 */
#ifndef LBM_NN_H
#define LBM_NN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Forward convolution with bias and optional ReLU, on the matrix cores
 * (BF16 operands, FP32 accumulation).  x: bf16 view (ldx % 4 == 0, 8-byte
 * aligned), ci and co multiples of 16; w: bf16 [27][co][ci]; bias: FP32
 * [co]; y: a bf16 view (y_fp32 = 0) or an FP32 view (y_fp32 = 1), ldy % 4 == 0.
 * The input gradient of a convolution is this same call on the output
 * gradient with the weights of nn_weights_flip. */
int nn_conv3d_fwd(const uint16_t *x, int32_t ldx, const uint16_t *w, const float *bias, void *y, int32_t ldy,
                  int32_t y_fp32, int32_t relu, int32_t nb, int32_t d, int32_t h, int32_t w_, int32_t ci,
                  int32_t co, void *stream);

/* wt[26 - t][ci][co] = w[t][co][ci] (bf16): the weights of the adjoint
 * convolution (gradient with respect to the input). */
int nn_weights_flip(const uint16_t *w, uint16_t *wt, int32_t ci, int32_t co, void *stream);

/* Weight and bias gradients: dw[t][co][ci] = sum_p dy[p][co] x[p + d_t][ci],
 * db[co] = sum_p dy[p][co] (FP32 outputs, overwritten).  x, dy: bf16 views
 * (ci, co multiples of 16).  work: FP32 scratch of at least
 * nn_bwd_weight_work(nb, d, h, w_, ci, co) floats.  The sums run in a fixed
 * order: the result does not depend on the launch. */
int64_t nn_bwd_weight_work(int32_t nb, int32_t d, int32_t h, int32_t w_, int32_t ci, int32_t co);
int nn_conv3d_bwd_weight(const uint16_t *x, int32_t ldx, const uint16_t *dy, int32_t lddy, float *dw, float *db,
                         float *work, int64_t work_floats, int32_t nb, int32_t d, int32_t h, int32_t w_,
                         int32_t ci, int32_t co, void *stream);

/* out = bf16(relu ? dy * (y > 0) : dy): the gradient at a convolution's
 * output made ready for its backward calls.  dy: FP32 view, y: bf16 view
 * (the layer's output), out: bf16 view; p positions, c channels. */
int nn_relu_bwd_cast(const float *dy, int32_t lddy, const uint16_t *y, int32_t ldy, uint16_t *out, int32_t ldo,
                     int64_t p, int32_t c, int32_t relu, void *stream);

/* 2 x 2 x 2 average pooling of a bf16 view (d, h, w_: input sizes, even)
 * and its adjoint on FP32 gradients: dx (+)= dy / 8 on each child
 * (accumulate = 1 adds to dx, 0 overwrites). */
int nn_pool2_fwd(const uint16_t *x, int32_t ldx, uint16_t *y, int32_t ldy, int32_t nb, int32_t d, int32_t h,
                 int32_t w_, int32_t c, void *stream);
int nn_pool2_bwd(const float *dy, int32_t lddy, float *dx, int32_t lddx, int32_t accumulate, int32_t nb, int32_t d,
                 int32_t h, int32_t w_, int32_t c, void *stream);

/* Nearest 2x upsampling of a bf16 view (d, h, w_: input sizes) and its
 * adjoint on FP32 gradients: dx = sum of dy over the 8 children. */
int nn_up2_fwd(const uint16_t *x, int32_t ldx, uint16_t *y, int32_t ldy, int32_t nb, int32_t d, int32_t h, int32_t w_,
               int32_t c, void *stream);
int nn_up2_bwd(const float *dy, int32_t lddy, float *dx, int32_t lddx, int32_t nb, int32_t d, int32_t h, int32_t w_,
               int32_t c, void *stream);

/* Weighted mean-square loss L = sum_c cw[c] mean_p (pred - target)^2 over
 * p positions and c channels and its gradient dpred (FP32 view,
 * overwritten).  loss: FP64 device array of at least 257 elements; loss[0]
 * receives L (summed in a fixed order), the rest is scratch.  pred, target:
 * FP32 views (ldp, ldt); cw: FP32 [c]. */
int nn_mse(const float *pred, int32_t ldp, const float *target, int32_t ldt, const float *cw, float *dpred,
           int32_t lddp, double *loss, int64_t p, int32_t c, void *stream);

/* One Adam update of n FP32 parameters from their gradients (step t >= 1,
 * bias-corrected moments m, v kept by the caller) and their bf16 copy for
 * the matrix cores. */
int nn_adam(float *param, const float *grad, float *m, float *v, uint16_t *param_bf16, int64_t n, float lr, float b1,
            float b2, float eps, int32_t t, void *stream);

/* y = bf16(x), n elements (contiguous). */
int nn_to_bf16(const float *x, uint16_t *y, int64_t n, void *stream);

/* The surrogate's geometry feature: Euclidean distance (FP32) from each of
 * the d x h x w sites of a periodic lattice (x fastest) to the nearest site
 * with solid[s] != 0, exact wherever that site lies within +-radius along
 * every axis, else radius sqrt(3).  Separable: the distance along x, then
 * minima over y and z of the squared distances.  work: FP32 scratch of 2
 * d h w floats. */
int nn_solid_distance(const uint8_t *solid, float *work, float *dist, int32_t d, int32_t h, int32_t w_, int32_t radius,
                      void *stream);

/* The surrogate's input: bf16 channels [solid, rho_a / (rho_a + rho_b) on
 * fluid sites (else 0), dist / dist_scale, 0, ...] for p positions, c >= 3
 * channels at stride ldx >= c. */
int nn_features(const uint8_t *solid, const double *rho_a, const double *rho_b, const float *dist, float dist_scale,
                uint16_t *x, int32_t ldx, int32_t c, int64_t p, void *stream);

/* The warm state from the surrogate's output (FP32 view out, ldo >= 5:
 * [ux, uy, uz, d rho_a, d rho_b] in units of u_scale g / nu_mix and
 * rho_scale), at fluid sites: u = out * u_scale * g / nu_mix with nu_mix =
 * phi nu_a + (1 - phi) nu_b of the initial fraction phi (Eqs. 5-6), rho =
 * max(rho0 + rho_scale * out, floor), then each density rescaled so that
 * its sum over fluid sites equals that of rho0 (FP64 sums in a fixed
 * order); zero on solid sites.  u: 3p doubles (component-major), rho_a,
 * rho_b: p doubles; work: FP64 scratch of at least 4096 doubles. */
int nn_decode_fields(const float *out, int32_t ldo, const uint8_t *solid, const double *rho_a0, const double *rho_b0,
                     double nu_a, double nu_b, double g, float u_scale, float rho_scale, double floor, double *u,
                     double *rho_a, double *rho_b, double *work, int64_t p, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* LBM_NN_H */
