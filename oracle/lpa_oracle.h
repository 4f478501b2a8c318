/*
 * lpa_oracle.h -- plain FP64 CPU oracle for multi-sensor HDR reconstruction by
 * local polynomial approximation (LPA) with ICI scale selection.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load or call this library.  It shares
 * no source with the GPU library and never serves the product path.
 *
 * What it computes (Kronander et al., "A Unified Framework for Multi-Sensor
 * HDR Video Reconstruction", arXiv 1308.4908):
 *   - per-sample radiance estimate, Sec. 6 eq. (Efsi), and its variance
 *     estimate, Sec. 6.1 eq. (varianceestiamte); saturated samples excluded
 *     (Sec. 6.1, last paragraph);
 *   - sample positions in the reference plane through the affine T_s
 *     (Sec. 4.2) and output positions through the output map (Sec. 3/4.2);
 *   - the M-th order local polynomial model with the tril basis (Sec. 5.1);
 *   - the localized-likelihood weighted least squares fit, eq. (wlsqe),
 *     with an isotropic Gaussian window H = hI (Sec. 5.2, Sec. 5.3.1);
 *   - the "invertible normal matrix" scale rule of Sec. 5.3.1 made numeric;
 *   - ICI (intersection of confidence intervals) selection among several
 *     window radii.  ICI is not in the paper; it is the rule of Goldenshluger
 *     and Nemirovski (1997) and Katkovnik (1999) from the LPA literature the
 *     paper cites for its window family.
 *
 * Readings taken where the paper is silent or inconsistent (each one is listed
 * with its reason in the design notes of the repository):
 *   R1  weight = window * inverse VARIANCE (the likelihood of Sec. 5.2 is
 *       Gaussian, so the residual is divided by sigma^2);
 *   R2  window exp(-|d|^2 / h) (the explicit Gaussian of Sec. 5.3.1), made to
 *       vanish at the support radius r: K = exp(-|d|^2/h) - exp(-r^2/h) for
 *       |d| < r, else 0; default h = 2 r^2 / 9; the normalisation constant is
 *       dropped (it cancels in the estimate and in its variance);
 *   R3  radii r and h are in reference-plane units; green uses r*kappa_G and
 *       h*kappa_G^2 (Sec. 5.3.1 suggests kappa_G = 2^-1/4; default 1);
 *   R4  sensor pixel centres sit at integer (col, row);
 *   R5  a sample is masked iff y >= saturation;
 *   R6  exposure = n_s t_s, non-uniformity a = 1, scalar bias frame; the shot
 *       term of the variance is clamped at 0 when y < b;
 *   R7  "invertible": N >= n and rho >= tau_inv, where rho is the smallest
 *       Cholesky pivot of the Jacobi-equilibrated normal matrix;
 *   R8  ICI with inclusive ties, Gamma-sigma intervals, sigma^2 the exact
 *       variance of the linear estimator (sandwich e0' A^-1 B A^-1 e0);
 *   R9  if no scale is valid at order M, fall back to order M-1, ..., 0 on the
 *       same samples; if nothing is valid the output is NaN.
 */
#ifndef LPA_ORACLE_H
#define LPA_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MAX_SENSORS 8
#define ORC_MAX_SCALES 8

/* CFA pattern: colour of the 2x2 cell, read row-major from (0,0). */
enum { ORC_CFA_RGGB = 0, ORC_CFA_BGGR = 1, ORC_CFA_GRBG = 2, ORC_CFA_GBRG = 3 };

typedef struct {
  int32_t width, height; /* sensor size in pixels                           */
  int32_t cfa;           /* ORC_CFA_*                                        */
  double affine[6];      /* X = a0*x + a1*y + a2, Y = a3*x + a4*y + a5       */
  double exposure;       /* n_s * t_s                                        */
  double gain;           /* g_s [DN / e-]                                    */
  double read_sigma;     /* sqrt(Var[r_s]) [DN]                              */
  double black_level;    /* b_s [DN]                                         */
  double saturation;     /* masked iff y >= saturation [DN]                  */
} orc_sensor;

typedef struct {
  int32_t out_w, out_h;
  double out_affine[6];  /* output pixel (u = col, v = row) -> reference plane */
  int32_t order;         /* M in {0, 1, 2}                                     */
  int32_t n_scales;      /* 1..ORC_MAX_SCALES, radii ascending                 */
  double radii[ORC_MAX_SCALES];
  double h[ORC_MAX_SCALES]; /* <= 0 selects the default 2 r^2 / 9              */
  double gamma;          /* ICI interval half-width in standard deviations     */
  double green_ratio;    /* kappa_G                                            */
  double tau_inv;        /* validity threshold on the equilibrated pivot       */
  int32_t exhaustive;    /* 1: visit every sample of every sensor (no box)     */
} orc_params;

/* Per (pixel, channel, scale, order) diagnostics. */
typedef struct {
  double yhat;   /* C0 of the fit                                 */
  double var;    /* variance of C0 (sandwich formula)             */
  double rho;    /* smallest equilibrated Cholesky pivot (0 if not SPD) */
  double c1x, c1y; /* gradient C1 (orders >= 1), else 0           */
  double l1f;    /* sum_k |a_k f_k| with C0 = sum_k a_k f_k: the size of the terms
                    the estimate sums (its rounding-error scale) */
  double sens_y; /* first-order bound on |dC0| per unit relative perturbation of
                    every moment term: |g|'|b|abs + |g|'|A|abs|C|, with g = A^-1 e0,
                    |A|abs = sum w |phi phi'|, |b|abs = sum w |f phi| */
  double sens_v; /* same for var(C0): 2 |B g|' |A^-1| |A|abs |g| + |g|' |B|abs |g| */
  int32_t n;     /* number of samples with positive window weight */
  int32_t valid; /* n >= basis size and rho >= tau_inv            */
} orc_fit;

/*
 * Reconstruct the listed output pixels.
 *   raw[s]      : sensor s digital values as doubles, row-major width*height
 *   pixels      : n_pixels (u, v) pairs; NULL means the whole output grid in
 *                 row-major order (n_pixels must then equal out_w*out_h)
 *   rgb         : n_pixels * 3 outputs (R, G, B); NaN where nothing is valid
 *   scale_map   : optional, n_pixels * 3 bytes: order_used << 4 | scale index,
 *                 0xFF when nothing is valid
 *   margin      : optional, n_pixels * 3: smallest ICI decision margin
 *                 |U - L| / (Gamma * sqrt(var)) over the steps taken (+Inf if
 *                 fewer than two valid scales)
 *   gap         : optional, n_pixels * 3: smallest |U - L| over those steps
 *                 (radiance units; +Inf if fewer than two valid scales)
 *   fits        : optional, n_pixels * 3 * n_scales * 3 entries, index
 *                 ((p * 3 + c) * n_scales + m) * 3 + order
 * Returns 0 on success, a negative value on invalid arguments.
 */
int orc_reconstruct(const orc_sensor* sensors, int32_t n_sensors, const double* const* raw,
                    const orc_params* params, const int32_t* pixels, int64_t n_pixels, double* rgb,
                    uint8_t* scale_map, double* margin, double* gap, orc_fit* fits);

/* Radiance estimate and variance estimate of one sample (Sec. 6, 6.1).
 * Returns 1 if the sample is usable (not saturated), 0 if masked. */
int orc_sample_radiance(const orc_sensor* sensor, double y, double* f_hat, double* var_hat);

/* Channel (0 = R, 1 = G, 2 = B) of sensor pixel (x, y) for a CFA pattern. */
int orc_cfa_channel(int32_t cfa, int32_t x, int32_t y);

/* The ICI rule on given per-scale estimates (used by the unit tests on worked
 * examples).  valid[m] != 0 marks a usable scale.  Returns the chosen scale or
 * -1 if none is valid; *margin_out receives the smallest decision margin and
 * *gap_out the smallest |U - L| (either may be NULL). */
int orc_ici_select(int32_t n_scales, const double* yhat, const double* var, const int32_t* valid,
                   double gamma, double* margin_out, double* gap_out);

#ifdef __cplusplus
}
#endif
#endif
