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
 *   R6  exposure = n_s t_s; without calibration frames the non-uniformity
 *       is a = 1 and the bias frame a scalar; the shot term of the variance is
 *       clamped at 0 when y < b;
 *   R7  "invertible": N >= n and rho >= tau_inv, where rho is the smallest
 *       Cholesky pivot of the Jacobi-equilibrated normal matrix;
 *   R8  ICI with inclusive ties, Gamma-sigma intervals, sigma^2 the exact
 *       variance of the linear estimator (sandwich e0' A^-1 B A^-1 e0);
 *   R9  if no scale is valid at order M, fall back to order M-1, ..., 0 on the
 *       same samples; if nothing is valid the output is NaN;
 *   R23 per-pixel calibration frames (bias b_i, non-uniformity a_i, readout
 *       variance, saturation frame; Sec. 6) are optional per sensor and frame
 *       kind; a defect mask (not in the paper) excludes pixels like saturation.
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
  /* Optional per-pixel calibration frames (Sec. 6), row-major width*height;
   * NULL selects the scalar above (R23):
   *   bias      bias frame b_{s,i} [DN]                  (for black_level)
   *   prnu      photo-response non-uniformity a_{s,i} > 0 (for a = 1)
   *   read_var  readout variance Var[r_{s,i}] [DN^2]     (for read_sigma^2)
   *   sat       saturation frame [DN]: masked iff y >= sat_i (for saturation)
   *   defect    nonzero: a defective pixel, never used                     */
  const double* bias;
  const double* prnu;
  const double* read_var;
  const double* sat;
  const uint8_t* defect;
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
/* The same for sensor pixel i = row * width + col, with its calibration
 * frames where the sensor has them. */
int orc_sample_radiance_at(const orc_sensor* sensor, int64_t i, double y, double* f_hat, double* var_hat);

/* Channel (0 = R, 1 = G, 2 = B) of sensor pixel (x, y) for a CFA pattern. */
int orc_cfa_channel(int32_t cfa, int32_t x, int32_t y);

/* The ICI rule on given per-scale estimates (used by the unit tests on worked
 * examples).  valid[m] != 0 marks a usable scale.  Returns the chosen scale or
 * -1 if none is valid; *margin_out receives the smallest decision margin and
 * *gap_out the smallest |U - L| (either may be NULL). */
int orc_ici_select(int32_t n_scales, const double* yhat, const double* var, const int32_t* valid,
                   double gamma, double* margin_out, double* gap_out);

/* ---------------------------------------------------------------------------
 * Adaptive anisotropic LPA with colour-channel correlation (CALPA), Sec. 5.4
 * and Sec. 5.5.  Three stages:
 *   1. orc_gradients: the gradient C1 of an isotropic order >= 1 fit of the G
 *      channel at every output pixel (Sec. 5.4 first step; Sec. 5.5: G only);
 *   2. orc_steering: per output pixel, the local gradient matrix over the
 *      (2q+1)^2 neighbouring output pixels, its two singular values s1 >= s2
 *      and directions, and from them the steering matrix
 *      C = gamma U diag(sigma, 1/sigma) U^T, sigma = (s1 + l1) / (s2 + l1),
 *      gamma = ((s1 s2 + l2) / M)^alpha, elongated along the edge;
 *   3. orc_reconstruct_steered: the LPA-ICI reconstruction of all channels
 *      with the window exp(-d^T C d / h) - exp(-r^2 / h) on the ellipse
 *      d^T C d < r^2 (C = I gives orc_reconstruct exactly).
 * Readings (each listed with its reason in the design notes):
 *   R18 the window exponent is d^T C d / h, not d^T (hC)^-1 d: with C built as
 *       Sec. 5.4 writes it (large eigenvalue sigma*gamma across the edge), the
 *       inverse would widen the window across edges, against the section's
 *       stated intent and the steering kernels it cites;
 *   R19 Lambda = Delta, and U Lambda U^T (the transpose the text omits);
 *   R20 the gradient analysis window w is uniform over the (2q+1)^2 output
 *       pixels around j that lie in the output grid; M is their number;
 *       pixels whose gradient fit is invalid contribute a zero gradient;
 *   R21 the eigenvalues gamma*sigma and gamma/sigma of C are clamped to
 *       [1/kappa^2, kappa^2] so the support stays within kappa r of X_j
 *       (the paper states no bound; a tile-staged implementation needs one);
 *   R22 gradients come from the G channel at radius grad_radius (times
 *       kappa_G, like every G window), order grad_order, isotropic window.
 * ------------------------------------------------------------------------- */
typedef struct {
  double alpha;        /* structure sensitivity (>= 0)                          */
  double lambda1;      /* elongation regulariser (paper: 1)                     */
  double lambda2;      /* scaling regulariser (paper: 0.001)                    */
  double grad_radius;  /* radius of the gradient fit (reference units)          */
  double grad_h;       /* its window parameter; <= 0 selects 2 r^2 / 9          */
  double max_stretch;  /* kappa >= 1 (R21)                                      */
  int32_t grad_order;  /* 1 or 2                                                */
  int32_t grad_halfwin;/* q >= 0: analysis window of (2q+1)^2 output pixels     */
} orc_adapt;

/* Stage 1.  grad: 2 doubles per listed pixel (reference-plane units, zero
 * where the fit is invalid); valid: optional, 1 per pixel.  pixels == NULL
 * means the whole output grid in row-major order.  Returns 0 or < 0. */
int orc_gradients(const orc_sensor* sensors, int32_t n_sensors, const double* const* raw,
                  const orc_params* params, const orc_adapt* adapt, const int32_t* pixels,
                  int64_t n_pixels, double* grad, int32_t* valid);

/* Stage 2 from a gradient plane covering the whole output grid (row-major,
 * 2 doubles per pixel).  C: 3 doubles per listed pixel (cxx, cxy, cyy);
 * diag: optional, 5 per pixel (s1, s2, theta, sigma, gamma). */
int orc_steering(const orc_params* params, const orc_adapt* adapt, const double* grad_plane,
                 const int32_t* pixels, int64_t n_pixels, double* C, double* diag);

/* Stage 3 with given steering matrices (3 doubles per listed pixel; NULL
 * means the identity).  Outputs as orc_reconstruct. */
int orc_reconstruct_steered(const orc_sensor* sensors, int32_t n_sensors, const double* const* raw,
                            const orc_params* params, const double* C, const int32_t* pixels,
                            int64_t n_pixels, double* rgb, uint8_t* scale_map, double* margin,
                            double* gap, orc_fit* fits);

/* Temporal (3-D) LPA (Sec. 9 names the extension of the supports from space to
 * space and time as future work; its form here is a reading of our own):
 *   T1 n_times frames of the rig at integer times t = 0, -1, ..., -(n_times - 1)
 *      (causal: the output is the estimate at t = 0); raw[t * n_sensors + s]
 *      is sensor s's frame at time -t, all through the same sensor maps and
 *      noise model;
 *   T2 the window of a sample at time -t is the spatial window (R3) times
 *      exp(-t^2 / h_t[m]), one temporal scale per radius, so that ICI selects
 *      a spatio-temporal scale; h_t[m] = 0 keeps only t = 0;
 *   T3 the local model is constant in t (the basis is the spatial one): the
 *      support, not the polynomial, extends to time;
 *   T4 no motion compensation: a scene that moves is handled by the scale
 *      selection, which shrinks the support where frames disagree.
 * Outputs as orc_reconstruct. */
#define ORC_MAX_TIMES 16
int orc_reconstruct_temporal(const orc_sensor* sensors, int32_t n_sensors, int32_t n_times,
                             const double* const* raw, const orc_params* params, const double* h_t,
                             const int32_t* pixels, int64_t n_pixels, double* rgb, uint8_t* scale_map,
                             double* margin, double* gap, orc_fit* fits);

#ifdef __cplusplus
}
#endif
#endif
