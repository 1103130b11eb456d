/*
 * bbsur -- learned surrogate of the transcranial FDTD solve: a 3D Fourier
 * neural operator mapping per-cell speed, density and incident-field phase of
 * an n^3 domain to the log peak-pressure map, trained on FDTD solves of libbbfd
 * and falling back to them (the FDTD solve stays the reference for its error).
 *
 * Every contraction (lifting, pointwise layers, the truncated Fourier
 * transforms written as matrix products, projection, and all their gradients)
 * runs on the gfx950 BF16 matrix cores with FP32 accumulation: operands are
 * FP32 in memory and rounded to BF16 as they are staged.  Element-wise steps
 * (GELU, per-mode complex channel mixing, loss, Adam) run in FP32.
 *
 * Network (n^3 volumes, x fastest, channels outermost per sample):
 *   h0 = W_lift x + b_lift                          cin -> width
 *   z_l = S_l(h_{l-1}) + W_l h_{l-1} + b_l, h_l = GELU(z_l),  l = 1..layers
 *   y = W_proj h_layers + b_proj                    width -> 1
 * S_l keeps Fourier modes kx in [0, mx), ky in {0..my-1, -my..-1}, kz in
 * {0..mz-1, -mz..-1} of the real FFT of its input, multiplies each mode by a
 * complex width x width matrix and transforms back (inverse real FFT of the
 * zero-padded spectrum).  GELU(z) = z/2 (1 + erf(z / sqrt 2)).
 *
 * Flat FP32 parameter vector, in order: W_lift [width][cin], b_lift [width];
 * per layer: R [2][Q][width][width] (real plane then imaginary plane, Q =
 * mx * 2my * 2mz modes ordered (kz, ky, kx) with kx fastest, [q][c][o]),
 * W [width][width] ([out][in]), b [width]; W_proj [1][width], b_proj [1].
 *
 * Conventions as libbbfd: caller-owned device buffers ("dev"), HIP stream
 * handles, return 0 or a negative BBFD_E* code (bbfd.h), bbfd_last_error().
 */
#ifndef BBSUR_H
#define BBSUR_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t n;      /* cells per axis of the cubic domain, a multiple of 8 (8 .. 256) */
  int32_t cin;    /* input channels */
  int32_t width;  /* channels of the hidden layers */
  int32_t layers; /* Fourier layers */
  int32_t mx, my, mz; /* kept modes per axis (mx <= n/2, 2my <= n, 2mz <= n) */
  float loss_focus;   /* training loss weight: w = 1 + loss_focus * exp(target) (>= 0) */
} bbsur_config;

typedef struct bbsur_model bbsur_model;

int bbsur_create(const bbsur_config *cfg, bbsur_model **out);
void bbsur_destroy(bbsur_model *model);
/* Parameter count and the device workspace a forward/backward pass on
   `batch` samples needs. */
int bbsur_sizes(const bbsur_model *model, int32_t batch, uint64_t *n_params,
                uint64_t *workspace_bytes);
/* Deterministic initialisation from seed (host RNG, copied to params). */
int bbsur_init_params(const bbsur_model *model, float *params, uint64_t seed, void *stream);
/* y (dev, [batch][n^3]) = network(x (dev, [batch][cin][n^3])). */
int bbsur_forward(const bbsur_model *model, const float *params, const float *x, float *y,
                  int32_t batch, void *workspace, uint64_t workspace_bytes, void *stream);
/* Gradient of sum(dy * network(x)) with respect to the parameters (overwrites
   grad, n_params floats); the forward pass is recomputed. */
int bbsur_backward(const bbsur_model *model, const float *params, const float *x,
                   const float *dy, float *grad, int32_t batch, void *workspace,
                   uint64_t workspace_bytes, void *stream);
/* One Adam step on the weighted mean squared error to target ([batch][n^3]),
   mean over cells of w (y - target)^2 with w = 1 + loss_focus exp(target)
   (targets are logs of normalised pressure, so the weight grows with the
   pressure the target stands for; loss_focus = 0 is the plain MSE):
   forward, loss (written to loss_dev[0]), backward, update of params with
   moments m, v (n_params floats each, zero at step 1).  step counts from 1. */
int bbsur_train_step(const bbsur_model *model, float *params, float *grad, float *m, float *v,
                     int32_t step, float lr, const float *x, const float *target, int32_t batch,
                     float *loss_dev, void *workspace, uint64_t workspace_bytes, void *stream);
/* Input channels of one sample from a material map (dev uint8 [cells]), a
   per-material table of n_table rows (dev float2: c/c_w - 1, rho/rho_w - 1;
   indices beyond it read as 0) and a complex incident field (dev complex64
   [cells]): x = [c', rho', cos phase, sin phase] ([4][cells]). */
int bbsur_features(const uint8_t *mat, const float *table, int32_t n_table,
                   const float *field_re_im, float *x, int64_t cells, void *stream);
/* Building block, exposed for tests: C = alpha A B + beta C (+ bias[m]) with
   strided operands (A FP32 [M][K] at a_strides = {batch, m, k}, B FP32 [K][N]
   at b_strides = {batch, k, n}, C at c_strides = {batch, m, n}) on the BF16
   matrix cores. */
int bbsur_gemm(const float *A, const int64_t *a_strides, const float *B, const int64_t *b_strides,
               float *C, const int64_t *c_strides, const float *bias, int32_t M, int32_t N,
               int32_t K, int32_t batch, float alpha, float beta, void *stream);

#ifdef __cplusplus
}
#endif
#endif
