/*
 * stfd_fno.h - C ABI of the learned warm start: a small spectral-convolution
 * network that maps the potential and the initial datum of a problem to an
 * initial guess x_0 for the preconditioned CG of stfd_pcg_solve (the paper's
 * solver is unchanged; a cold start x_0 = 0 stays the fallback).
 *
 * Network (FP32, channels innermost, tensors [batch][i_2][i_1][channel]):
 *   a_0 = x W_P + b_P                                  (c_in -> width, pointwise)
 *   z_l = a_l W_l + b_l + K_l(a_l),  a_{l+1} = GELU(z_l) for l < layers-1, a_L = z_{L-1}
 *   y   = GELU(a_L Q_1 + q_1) Q_2 + q_2                 (width -> proj -> c_out)
 * GELU(z) = z Phi(z) (exact, erf form).  Spectral convolution of one channel
 * field h (H x W):
 *   h_hat[k1,k2] = sum_{i1,i2} h[i2,i1] exp(-2 pi i (k1 i1 / W + k2 i2 / H)),
 *     k1 in [0, modes1), k2 in [-modes2/2, modes2/2)
 *   g_hat[k1,k2,o] = sum_c h_hat[k1,k2,c] R[k1,k2,c,o]          (complex weights)
 *   K(h)[i2,i1,o] = 1/(H W) sum_{k1,k2} w_k1 Re(g_hat[k1,k2,o] exp(+2 pi i (...))),
 *     w_0 = 1, w_k1 = 2 for k1 > 0 (half spectrum along i_1)
 * The truncated transforms are dense GEMMs with precomputed DFT matrices.
 *
 * Parameters: one flat FP32 array, in this order:
 *   W_P [c_in][width], b_P [width],
 *   per layer: W_l [width][width], b_l [width],
 *              R_l real [k2][k1][c][o], R_l imag [k2][k1][c][o]  (k2 index j = k2 mod modes2),
 *   Q_1 [width][proj], q_1 [proj], Q_2 [proj][c_out], q_2 [c_out].
 * Initialisation from `seed` (SplitMix64 uniforms): weights U(-1/sqrt(fan_in), 1/sqrt(fan_in)),
 * spectral weights U(0, 1) / (width * width), biases 0.
 *
 * Conventions: *_dev are device pointers owned by the caller; the handle owns its
 * parameters, gradients, Adam moments and activation workspace (sized for
 * max_batch at creation).  Calls are stream-ordered; a handle is used by one
 * stream at a time.  Every function returns a stfd_status (include/stfd.h).
 */
#ifndef STFD_FNO_H
#define STFD_FNO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct stfd_fno stfd_fno;

typedef struct {
  int H, W;        /* spatial grid (i_2, i_1) */
  int c_in;        /* input channels */
  int width;       /* hidden channels */
  int modes1;      /* retained frequencies along i_1 (0..modes1-1), <= W/2 + 1 */
  int modes2;      /* retained frequencies along i_2 (-modes2/2..modes2/2-1), even, <= H */
  int layers;      /* spectral layers */
  int proj;        /* hidden width of the projection */
  int c_out;       /* output channels */
  int max_batch;
  uint64_t seed;
} stfd_fno_desc;

/* Errors: STFD_EINVAL (non-positive sizes, modes out of range), STFD_ENOMEM, STFD_EHIP. */
int stfd_fno_create(const stfd_fno_desc *desc, stfd_fno **out);
int stfd_fno_num_params(const stfd_fno *net, int64_t *n);
/* Host copies of the parameters / of the gradients of the last backward, and parameter upload. */
int stfd_fno_get_params(const stfd_fno *net, float *host);
int stfd_fno_set_params(stfd_fno *net, const float *host);
int stfd_fno_get_grads(const stfd_fno *net, float *host);
/* y = net(x); x_dev [batch][H][W][c_in], y_dev [batch][H][W][c_out].  Keeps the activations
 * of this batch for stfd_fno_backward.  Errors: STFD_EINVAL (batch outside [1, max_batch]). */
int stfd_fno_forward(stfd_fno *net, const float *x_dev, float *y_dev, int batch, void *stream);
/* Gradients of sum(dy * y) with respect to every parameter (overwritten in the handle's
 * gradient buffer) for the batch of the last forward; dx_dev (may be NULL) receives the
 * gradient with respect to x. */
int stfd_fno_backward(stfd_fno *net, const float *dy_dev, float *dx_dev, int batch, void *stream);
/* Relative l2 loss (1/batch) sum_b ||y_b - t_b|| / ||t_b|| over n values per sample, and its
 * gradient dy (device, may be NULL).  *loss (host) is written after the stream synchronises. */
int stfd_fno_rel_l2(const float *y_dev, const float *t_dev, int64_t n, int batch, float *dy_dev,
                    float *loss, void *stream);
/* One Adam step (Kingma & Ba) on all parameters with the current gradients; step counter
 * kept in the handle (bias correction). */
int stfd_fno_adam_step(stfd_fno *net, float lr, float beta1, float beta2, float eps, void *stream);
/* e = y - t in FP64 (t may be NULL: e = y), n values. */
int stfd_fno_diff_f64(const float *y_dev, const float *t_dev, double *e_dev, int64_t n, void *stream);
/* Energy-norm loss of a prediction error, given e (FP64, [batch][n], n reals = interleaved complex
 * coefficients) and Ae = A e from stfd_matvec of a Hermitian positive definite operator A:
 * E_b = e_b^H A e_b, loss = (1/batch) sum_b sqrt(E_b / T_b) with T_b = t_energy_dev[b] (device; NULL:
 * 1), and dy_b = A e_b / (batch sqrt(E_b T_b)) (FP32, may be NULL), the gradient of the loss with
 * respect to the prediction.  energy_host (may be NULL) receives E_b; *loss is written after the
 * stream synchronises.  Relative errors in the energy norm are what CG minimises, so a warm start
 * trained this way is measured in the norm that decides its value. */
int stfd_fno_energy_loss(const double *e_dev, const double *Ae_dev, const double *t_energy_dev, int64_t n,
                         int batch, float *dy_dev, double *energy_host, float *loss, void *stream);
/* y (FP32, [batch][n]) -> x (FP64, [batch][n]) on the device: the network's complex output
 * channels (re, im pairs) become an initial guess for stfd_pcg_solve. */
int stfd_fno_to_f64(const float *y_dev, double *x_dev, int64_t n, void *stream);
void stfd_fno_destroy(stfd_fno *net);

#ifdef __cplusplus
}
#endif
#endif /* STFD_FNO_H */
