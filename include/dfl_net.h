/* Start-field network of the deflation subspace: the kernels that generate,
 * run and train a small 4D convolutional network whose outputs replace the
 * random start fields of the subspace generation (section 5.3), and the
 * inverse iteration (eq. (5.1)) that produces its training targets.
 *
 * The paper has no network; what is computed is stated with each call. The
 * network reads the context's gauge field, so every call takes a dfl_ctx
 * created by dfl_create (include/dfl.h) with the gauge field set where noted.
 *
 * Layouts (all device memory, owned by the caller, contiguous):
 *  - activation planes: float [C][V], sites in canonical order
 *    ((x0*L1 + x1)*L2 + x2)*L3 + x3;
 *  - noise: float [V][24], canonical site order;
 *  - weights of a 3^4 convolution: float [81][Cin][Cout], tap
 *    t = sum_mu (o_mu + 1) * 3^(3 - mu) for the offset o in {-1,0,1}^4;
 *    biases float [Cout];
 *  - quark fields: native FP64 fields as in include/dfl.h (dfl_pack).
 *
 * Errors as in include/dfl.h: negative codes, message from dfl_last_error().
 * All calls are stream-ordered on the context's stream unless stated.
 */
#ifndef DFL_NET_H
#define DFL_NET_H

#include "dfl.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Relaxed inverse iteration of eq. (5.1) in place on n native FP64 fields:
 * normalise each field, then `steps` times psi <- M_sap psi at the setup mass
 * m0_setup followed by normalisation (the first phase of dfl_setup). n is at
 * most Ns with FP64 Schwarz, max(Ns, nrhs_max) otherwise. Needs the gauge
 * field. Synchronises. DFL_ENONFINITE on non-finite input. */
int dfl_inverse_iteration(dfl_ctx *ctx, void *fields_dev, int n, int steps);

/* Network input planes x [96][V]: channel ((mu*3 + a)*3 + b)*2 + r holds the
 * real (r = 0) or imaginary (r = 1) part of U_mu(x)[a][b]; channels 72..95
 * copy the 24 noise values of the site. Needs the gauge field. */
int net_features(dfl_ctx *ctx, const float *noise_dev, float *x_dev);

/* Periodic 3^4 convolution:
 *   z[co][x] = b[co] + sum_{o in {-1,0,1}^4} sum_ci W[t(o)][ci][co] in[ci][x + o],
 * and a = silu(z) = z / (1 + exp(-z)) when a is not NULL. b may be NULL (no
 * bias). 1 <= cin <= 96, 1 <= cout <= 576; z and a must not overlap in. */
int conv4d_forward(dfl_ctx *ctx, const float *in_dev, int cin, const float *W_dev, const float *b_dev, int cout,
                   float *z_dev, float *a_dev);

/* conv4d_forward with BF16 operands: every input value and weight is rounded
 * to BF16 (nearest even) and the products are summed in FP32 on the matrix
 * cores; bias and activation in FP32. Per output, |z - z_exact| is at most
 * about 2^-7 sum_o sum_ci |W| |in| (two roundings of 2^-8 relative each).
 * For inference (the start fields of section 5.3); training uses the FP32
 * map. Needs L3 % 32 == 0 and L2 % 4 == 0 (DFL_EINVAL otherwise); the
 * context keeps a BF16 copy of the weights (at most 81 x 96 x 576 entries),
 * grown on first use (synchronises then). Channel limits and overlap rules
 * as conv4d_forward. */
int conv4d_forward_bf16(dfl_ctx *ctx, const float *in_dev, int cin, const float *W_dev, const float *b_dev,
                        int cout, float *z_dev, float *a_dev);

/* Backward of conv4d_forward for the gradient g [cout][V] of a loss with
 * respect to z: dW[t][ci][co] = sum_x in[ci][x + o_t] g[co][x] and
 * db[co] = sum_x g[co][x] (both overwritten, summed in a fixed order), and,
 * if din is not NULL, din[ci][x] = sum_o sum_co W[t(o)][ci][co] g[co][x - o],
 * multiplied by silu'(z_in[ci][x]) when z_in (the pre-activation that
 * produced `in`) is not NULL. Same channel limits as the forward call. */
int conv4d_backward(dfl_ctx *ctx, const float *in_dev, int cin, const float *W_dev, int cout, const float *g_dev,
                    float *dW_dev, float *db_dev, float *din_dev, const float *z_in_dev);

/* conv4d_backward without any allocation, for callers that cannot allocate
 * device memory (code under graph capture, serving loops, harnesses that
 * forbid hipMalloc). Same arguments, results and errors as conv4d_backward,
 * except that the weight-gradient partial sums live in a fixed device array of
 * 64 MiB that the library holds on every device it runs on until the process
 * ends (conv4d_backward grows a context buffer instead); when the default
 * chunking over the sites needs more, fewer and longer chunks are summed, so
 * dW may differ from conv4d_backward's by FP32 rounding. No call allocates.
 * The array is shared by every call on a device and keeps the last call's
 * contents: calls that overlap on one device (several streams, contexts or
 * threads) race and must be serialised by the caller. */
int conv4d_backward_noalloc(dfl_ctx *ctx, const float *in_dev, int cin, const float *W_dev, int cout,
                            const float *g_dev, float *dW_dev, float *db_dev, float *din_dev, const float *z_in_dev);

/* Ns native FP64 fields from the last layer's planes out [24*Ns][V]:
 * component c of field l is out[(l*12 + c)*2] + i out[(l*12 + c)*2 + 1]. */
int net_outputs_to_fields(dfl_ctx *ctx, const float *out_dev, int Ns, void *fields_dev);

/* The adjoint map for gradients: given dL/dconj(field_l) (native FP64), the
 * gradient of the real loss L with respect to the output planes, 2 Re and
 * 2 Im of it, into dout [24*Ns][V]. 1 <= Ns <= 24. */
int net_fields_grad_to_outputs(dfl_ctx *ctx, const void *grad_dev, int Ns, float *dout_dev);

/* Mean deficit (eq. (3.15)) of the K target fields t_k with respect to the
 * block-wise span of the Ns fields Psi over the context's deflation blocks:
 *   loss = (1/K) sum_k ||(1 - P) t_k||^2 / ||t_k||^2,
 * P the orthogonal projector onto span{Psi_l restricted to Lambda} on every
 * block Lambda (per block G = Psi^+ Psi, c_k = Psi^+ t_k, ||P t_k||^2 =
 * c_k^+ G^-1 c_k, by Cholesky in FP64). If grad is not NULL it receives
 * dL/dconj(Psi_l) = -sum_k (t_k - Psi y_k) y_l,k^* / (K ||t_k||^2),
 * y_k = G^-1 c_k (native FP64, Ns fields). 1 <= Ns, K <= 32 and Ns <= 12
 * |block|. loss is a host pointer; synchronises. DFL_ESINGULAR if the fields
 * are linearly dependent on some block, DFL_EINVAL for a zero target. */
int deficit_loss(dfl_ctx *ctx, const void *fields_dev, int Ns, const void *targets_dev, int K, double *loss,
                 void *grad_dev);

/* One Adam step (Kingma and Ba) on n FP32 parameters, t >= 1 the step count:
 *   m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
 *   theta -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps). */
int adam_update(dfl_ctx *ctx, float *theta_dev, const float *g_dev, float *m_dev, float *v_dev, long long n, int t,
                double lr, double b1, double b2, double eps);

#ifdef __cplusplus
}
#endif

#endif /* DFL_NET_H */
