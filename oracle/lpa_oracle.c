/*
 * lpa_oracle.c -- plain, slow, single-threaded FP64 oracle for LPA + ICI HDR
 * reconstruction from multi-sensor raw CFA data (arXiv 1308.4908).
 *
 * TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark are its only callers.  It shares no code
 * with the GPU library.  Each function cites the passage of the paper it
 * follows; readings R1..R9 are stated in lpa_oracle.h.
 *
 * Structure: for each output pixel, colour channel and window radius the
 * support set is collected (every unmasked sample of that channel from every
 * sensor whose reference-plane distance is below the radius), the weighted
 * normal equations of eq. (wlsqe) are formed explicitly as n x n matrices and
 * solved with a textbook Cholesky factorisation, for every order 0..M.  The
 * ICI rule then picks a radius per pixel and channel.  No tiling, no fusion,
 * no reuse between pixels.
 */
#include "lpa_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define NB_MAX 6 /* basis size for M = 2 */

/* Colour of a CFA site (Sec. 3: each sensor samples through a Bayer CFA).
 * Cell index = 2 * (row parity) + (column parity). */
int orc_cfa_channel(int32_t cfa, int32_t x, int32_t y) {
  static const int table[4][4] = {
      {0, 1, 1, 2}, /* RGGB */
      {2, 1, 1, 0}, /* BGGR */
      {1, 0, 2, 1}, /* GRBG */
      {1, 2, 0, 1}, /* GBRG */
  };
  if (cfa < 0 || cfa > 3) return -1;
  return table[cfa][2 * (y & 1) + (x & 1)];
}

/* Radiance estimate, Sec. 6 eq. (Efsi): f = (y - b_i) / (g t a_i n), with
 * exposure = n t.  Variance estimate, Sec. 6.1 eq. (varianceestiamte):
 * (g^2 t a_i n f + Var[r_i]) / (g^2 t^2 a_i^2 n^2), the shot term evaluated
 * at the noisy estimate f and clamped at zero (R6).  Samples at or above the
 * saturation frame are excluded (end of Sec. 6.1, R5), and so are defective
 * pixels.  Without calibration frames b_i, a_i, Var[r_i] and the saturation
 * level are the sensor's scalars, a_i = 1 (R23). */
int orc_sample_radiance_at(const orc_sensor* s, int64_t i, double y, double* f_hat, double* var_hat) {
  const int pix = i >= 0;
  if (pix && s->defect && s->defect[i]) return 0;
  const double sat = pix && s->sat ? s->sat[i] : s->saturation;
  if (y >= sat) return 0;
  const double b = pix && s->bias ? s->bias[i] : s->black_level;
  const double a = pix && s->prnu ? s->prnu[i] : 1.0;
  const double rv = pix && s->read_var ? s->read_var[i] : s->read_sigma * s->read_sigma;
  const double g = s->gain, e = s->exposure;
  const double f = (y - b) / (g * e * a);
  const double shot = f > 0.0 ? f : 0.0;
  *f_hat = f;
  *var_hat = (g * g * e * a * shot + rv) / (g * g * e * e * a * a);
  return 1;
}

int orc_sample_radiance(const orc_sensor* s, double y, double* f_hat, double* var_hat) {
  return orc_sample_radiance_at(s, -1, y, f_hat, var_hat);
}

/* ICI rule (not in the paper; R8).  Intervals [y_m - G sd_m, y_m + G sd_m] of
 * the valid scales are intersected in ascending order of radius; the last
 * scale whose running intersection is non-empty (L <= U) is chosen. */
int orc_ici_select(int32_t n_scales, const double* yhat, const double* var, const int32_t* valid,
                   double gamma, double* margin_out, double* gap_out) {
  double lo_run = -INFINITY, hi_run = INFINITY, margin = INFINITY, gap = INFINITY;
  int chosen = -1;
  for (int m = 0; m < n_scales; ++m) {
    if (!valid[m]) continue;
    const double sd = sqrt(var[m]);
    const double lo = yhat[m] - gamma * sd, hi = yhat[m] + gamma * sd;
    if (lo > lo_run) lo_run = lo;
    if (hi < hi_run) hi_run = hi;
    if (chosen >= 0) {
      const double mu = fabs(hi_run - lo_run) / (gamma * sd);
      if (mu < margin) margin = mu;
      if (fabs(hi_run - lo_run) < gap) gap = fabs(hi_run - lo_run);
    }
    if (lo_run <= hi_run)
      chosen = m;
    else
      break;
  }
  if (margin_out) *margin_out = margin;
  if (gap_out) *gap_out = gap;
  return chosen;
}

/* One sample of a support set: offset from the output position, radiance,
 * inverse variance and window value. */
typedef struct {
  double dx, dy, f, ivar, k;
} orc_sample;

typedef struct {
  orc_sample* v;
  int64_t n, cap;
} sample_list;

static int list_push(sample_list* l, orc_sample s) {
  if (l->n == l->cap) {
    int64_t cap = l->cap ? 2 * l->cap : 256;
    orc_sample* v = (orc_sample*)realloc(l->v, (size_t)cap * sizeof(orc_sample));
    if (!v) return -1;
    l->v = v;
    l->cap = cap;
  }
  l->v[l->n++] = s;
  return 0;
}

/* Apply an affine map [a0 a1 a2; a3 a4 a5] to (x, y). */
static void affine_apply(const double a[6], double x, double y, double* X, double* Y) {
  *X = a[0] * x + a[1] * y + a[2];
  *Y = a[3] * x + a[4] * y + a[5];
}

/* The samples of one frame (all sensors) in the window of (X, Y), channel c,
 * radius r, each window value times the frame's temporal factor kt; appended
 * to out. */
static int gather_frame(const orc_sensor* sensors, int n_sensors, const double* const* raw, double X, double Y,
                        int c, double r, double h, const double* C, int exhaustive, double kt, sample_list* out) {
  const double k_edge = exp(-r * r / h);
  /* the ellipse lies inside the disc of radius r / sqrt(smallest eigenvalue of C) */
  double reff = r;
  if (C) {
    const double lmin = 0.5 * (C[0] + C[2]) - sqrt(0.25 * (C[0] - C[2]) * (C[0] - C[2]) + C[1] * C[1]);
    if (!(lmin > 0.0)) return -1;
    reff = r / sqrt(lmin);
  }
  for (int s = 0; s < n_sensors; ++s) {
    const orc_sensor* S = &sensors[s];
    const double* a = S->affine;
    int x0 = 0, x1 = S->width - 1, y0 = 0, y1 = S->height - 1;
    if (!exhaustive) {
      /* Bounding box of the disc pulled back through T_s. */
      const double det = a[0] * a[4] - a[1] * a[3];
      const double i00 = a[4] / det, i01 = -a[1] / det, i10 = -a[3] / det, i11 = a[0] / det;
      const double px = i00 * (X - a[2]) + i01 * (Y - a[5]);
      const double py = i10 * (X - a[2]) + i11 * (Y - a[5]);
      const double wx = reff * sqrt(i00 * i00 + i01 * i01), wy = reff * sqrt(i10 * i10 + i11 * i11);
      const double bx0 = floor(px - wx) - 1, bx1 = ceil(px + wx) + 1;
      const double by0 = floor(py - wy) - 1, by1 = ceil(py + wy) + 1;
      if (bx1 < 0 || by1 < 0 || bx0 > S->width - 1 || by0 > S->height - 1) continue;
      if (bx0 > x0) x0 = (int)bx0;
      if (bx1 < x1) x1 = (int)bx1;
      if (by0 > y0) y0 = (int)by0;
      if (by1 < y1) y1 = (int)by1;
    }
    for (int y = y0; y <= y1; ++y) {
      for (int x = x0; x <= x1; ++x) {
        if (orc_cfa_channel(S->cfa, x, y) != c) continue;
        double f, var;
        const int64_t pi = (int64_t)y * S->width + x;
        if (!orc_sample_radiance_at(S, pi, raw[s][pi], &f, &var)) continue;
        double Xk, Yk;
        affine_apply(a, (double)x, (double)y, &Xk, &Yk);
        const double dx = Xk - X, dy = Yk - Y;
        const double d2 = C ? C[0] * dx * dx + 2.0 * C[1] * dx * dy + C[2] * dy * dy : dx * dx + dy * dy;
        if (!(d2 < r * r)) continue;
        const double k = (exp(-d2 / h) - k_edge) * kt;
        if (!(k > 0.0)) continue;
        orc_sample smp = {dx, dy, f, 1.0 / var, k};
        if (list_push(out, smp)) return -1;
      }
    }
  }
  return 0;
}

/* Support set of output position (X, Y) for channel c and radius r with
 * window parameter h (Sec. 5.2 supp W_H; Sec. 4.2 X = T_s(x); R2, R4, R5).
 * With a steering matrix C (3 entries, Sec. 5.4, R18) the window is
 * exp(-d'Cd / h) - exp(-r^2 / h) on the ellipse d'Cd < r^2; C == NULL is
 * the isotropic window (C = I).  Over n_times frames (raw[t * n_sensors + s]
 * is sensor s at time -t) the window of a sample at time -t is multiplied by
 * exp(-t^2 / h_t) (T2); with h_t = 0 only t = 0 belongs to the support. */
static int gather_support(const orc_sensor* sensors, int n_sensors, const double* const* raw,
                          double X, double Y, int c, double r, double h, const double* C,
                          int exhaustive, int n_times, double h_t, sample_list* out) {
  out->n = 0;
  for (int t = 0; t < n_times; ++t) {
    const double kt = t == 0 ? 1.0 : (h_t > 0.0 ? exp(-(double)t * t / h_t) : 0.0);
    if (!(kt > 0.0)) continue;
    if (gather_frame(sensors, n_sensors, raw + (size_t)t * n_sensors, X, Y, c, r, h, C, exhaustive, kt, out))
      return -1;
  }
  return 0;
}

/* Basis of the local polynomial model, Sec. 5.1:
 * [1, dx, dy, tril(d d^T)] with tril in lexicographic order (dx^2, dx dy, dy^2). */
static void basis(double dx, double dy, double phi[NB_MAX]) {
  phi[0] = 1.0;
  phi[1] = dx;
  phi[2] = dy;
  phi[3] = dx * dx;
  phi[4] = dx * dy;
  phi[5] = dy * dy;
}

/* Textbook Cholesky A = L L^T of an n x n SPD matrix.  Returns the smallest
 * pivot L_jj^2 (<= 0 if A is not positive definite; then L is incomplete). */
static double cholesky(int n, const double A[NB_MAX][NB_MAX], double L[NB_MAX][NB_MAX]) {
  double min_pivot = INFINITY;
  memset(L, 0, sizeof(double) * NB_MAX * NB_MAX);
  for (int j = 0; j < n; ++j) {
    double d = A[j][j];
    for (int k = 0; k < j; ++k) d -= L[j][k] * L[j][k];
    if (d < min_pivot) min_pivot = d;
    if (!(d > 0.0)) return min_pivot < 0.0 ? min_pivot : 0.0;
    L[j][j] = sqrt(d);
    for (int i = j + 1; i < n; ++i) {
      double t = A[i][j];
      for (int k = 0; k < j; ++k) t -= L[i][k] * L[j][k];
      L[i][j] = t / L[j][j];
    }
  }
  return min_pivot;
}

/* Solve (L L^T) x = rhs. */
static void chol_solve(int n, const double L[NB_MAX][NB_MAX], const double* rhs, double* x) {
  double z[NB_MAX];
  for (int i = 0; i < n; ++i) {
    double t = rhs[i];
    for (int k = 0; k < i; ++k) t -= L[i][k] * z[k];
    z[i] = t / L[i][i];
  }
  for (int i = n - 1; i >= 0; --i) {
    double t = z[i];
    for (int k = i + 1; k < n; ++k) t -= L[k][i] * x[k];
    x[i] = t / L[i][i];
  }
}

/* Weighted least squares fit of eq. (wlsqe) with n basis terms on a support
 * set: C = (Phi^T W Phi)^-1 Phi^T W f, W = diag(K_k / sigma_k^2) (R1).
 * Validity (R7) is judged on the Jacobi-equilibrated normal matrix.  The
 * variance of C0 is e0^T A^-1 B A^-1 e0 with B = Phi^T W Sigma W Phi, which
 * is sum K_k^2 / sigma_k^2 phi phi^T since Sigma = diag(sigma_k^2) (R8). */
static void fit_order(const sample_list* S, int n, double tau_inv, orc_fit* out) {
  double A[NB_MAX][NB_MAX] = {{0}}, B[NB_MAX][NB_MAX] = {{0}}, b[NB_MAX] = {0};
  /* sums of absolute terms (diagnostics: rounding sensitivity, not the fit) */
  double Aa[NB_MAX][NB_MAX] = {{0}}, Ba[NB_MAX][NB_MAX] = {{0}}, ba[NB_MAX] = {0};
  for (int64_t k = 0; k < S->n; ++k) {
    const orc_sample* s = &S->v[k];
    double phi[NB_MAX];
    basis(s->dx, s->dy, phi);
    const double w = s->k * s->ivar;
    const double w2 = s->k * s->k * s->ivar;
    for (int i = 0; i < n; ++i) {
      b[i] += w * s->f * phi[i];
      ba[i] += fabs(w * s->f * phi[i]);
      for (int j = 0; j < n; ++j) {
        A[i][j] += w * phi[i] * phi[j];
        B[i][j] += w2 * phi[i] * phi[j];
        Aa[i][j] += fabs(w * phi[i] * phi[j]);
        Ba[i][j] += fabs(w2 * phi[i] * phi[j]);
      }
    }
  }
  out->n = (int32_t)S->n;
  out->yhat = NAN;
  out->var = NAN;
  out->c1x = 0.0;
  out->c1y = 0.0;
  out->l1f = 0.0;
  out->sens_y = 0.0;
  out->sens_v = 0.0;
  out->rho = 0.0;
  out->valid = 0;

  double scale[NB_MAX];
  for (int i = 0; i < n; ++i) {
    if (!(A[i][i] > 0.0)) return;
    scale[i] = 1.0 / sqrt(A[i][i]);
  }
  double At[NB_MAX][NB_MAX] = {{0}};
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) At[i][j] = scale[i] * A[i][j] * scale[j];
  double L[NB_MAX][NB_MAX];
  const double rho = cholesky(n, At, L);
  out->rho = rho > 0.0 ? rho : 0.0;
  if (!(rho > 0.0)) return;

  /* C = D^-1/2 At^-1 D^-1/2 b and g = A^-1 e0 with D = diag(A). */
  double rhs[NB_MAX] = {0}, u[NB_MAX], C[NB_MAX], g[NB_MAX];
  for (int i = 0; i < n; ++i) rhs[i] = scale[i] * b[i];
  chol_solve(n, L, rhs, u);
  for (int i = 0; i < n; ++i) C[i] = scale[i] * u[i];
  for (int i = 0; i < n; ++i) rhs[i] = (i == 0) ? scale[0] : 0.0;
  chol_solve(n, L, rhs, u);
  for (int i = 0; i < n; ++i) g[i] = scale[i] * u[i];
  double var = 0.0;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) var += g[i] * B[i][j] * g[j];

  /* equivalent-kernel weights a_k = (g . phi_k) w_k, C0 = sum_k a_k f_k */
  double l1f = 0.0;
  for (int64_t k = 0; k < S->n; ++k) {
    const orc_sample* s = &S->v[k];
    double phi[NB_MAX];
    basis(s->dx, s->dy, phi);
    double gp = 0.0;
    for (int i = 0; i < n; ++i) gp += g[i] * phi[i];
    l1f += fabs(gp * s->k * s->ivar * s->f);
  }
  out->l1f = l1f;
  /* rounding sensitivities (see lpa_oracle.h) */
  double Ainv[NB_MAX][NB_MAX];
  for (int j = 0; j < n; ++j) {
    double e[NB_MAX], col[NB_MAX];
    for (int i = 0; i < n; ++i) e[i] = (i == j) ? scale[i] : 0.0;
    chol_solve(n, L, e, col);
    for (int i = 0; i < n; ++i) Ainv[i][j] = scale[i] * col[i];
  }
  double sy = 0.0, sv = 0.0, Bg[NB_MAX], Aag[NB_MAX];
  for (int i = 0; i < n; ++i) {
    double t = 0.0, q = 0.0;
    for (int j = 0; j < n; ++j) {
      sy += fabs(g[i]) * Aa[i][j] * fabs(C[j]);
      sv += fabs(g[i]) * Ba[i][j] * fabs(g[j]);
      t += B[i][j] * g[j];
      q += Aa[i][j] * fabs(g[j]);
    }
    sy += fabs(g[i]) * ba[i];
    Bg[i] = t;
    Aag[i] = q;
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) sv += 2.0 * fabs(Bg[i]) * fabs(Ainv[i][j]) * Aag[j];
  out->sens_y = sy;
  out->sens_v = sv;
  out->yhat = C[0];
  out->var = var;
  if (n >= 3) {
    out->c1x = C[1];
    out->c1y = C[2];
  }
  out->valid = (S->n >= n) && (rho >= tau_inv);
}

static int check_args(const orc_sensor* sensors, int32_t n_sensors, const double* const* raw,
                      const orc_params* P, const int32_t* pixels, int64_t n_pixels) {
  if (!sensors || !raw || !P) return -1;
  if (n_sensors < 1 || n_sensors > ORC_MAX_SENSORS) return -2;
  if (P->order < 0 || P->order > 2) return -3;
  if (P->n_scales < 1 || P->n_scales > ORC_MAX_SCALES) return -4;
  if (!pixels && n_pixels != (int64_t)P->out_w * P->out_h) return -5;
  for (int s = 0; s < n_sensors; ++s) {
    const orc_sensor* S = &sensors[s];
    const double det = S->affine[0] * S->affine[4] - S->affine[1] * S->affine[3];
    if (S->width < 1 || S->height < 1 || !(S->gain > 0) || !(S->exposure > 0) ||
        !(S->read_sigma > 0) || det == 0.0 || S->cfa < 0 || S->cfa > 3 || !raw[s])
      return -6;
    const int64_t np = (int64_t)S->width * S->height;
    for (int64_t i = 0; i < np; ++i)
      if ((S->prnu && !(S->prnu[i] > 0)) || (S->read_var && !(S->read_var[i] >= 0)) ||
          (S->bias && !isfinite(S->bias[i])) || (S->sat && isnan(S->sat[i])))
        return -7;
  }
  return 0;
}

static int reconstruct_impl(const orc_sensor* sensors, int32_t n_sensors, const double* const* raw,
                            int32_t n_times, const double* h_t, const orc_params* P, const double* Cpix,
                            const int32_t* pixels, int64_t n_pixels, double* rgb, uint8_t* scale_map,
                            double* margin, double* gap, orc_fit* fits);

int orc_reconstruct(const orc_sensor* sensors, int32_t n_sensors, const double* const* raw,
                    const orc_params* P, const int32_t* pixels, int64_t n_pixels, double* rgb,
                    uint8_t* scale_map, double* margin, double* gap, orc_fit* fits) {
  return reconstruct_impl(sensors, n_sensors, raw, 1, NULL, P, NULL, pixels, n_pixels, rgb, scale_map, margin, gap,
                          fits);
}

int orc_reconstruct_steered(const orc_sensor* sensors, int32_t n_sensors, const double* const* raw,
                            const orc_params* P, const double* C, const int32_t* pixels,
                            int64_t n_pixels, double* rgb, uint8_t* scale_map, double* margin,
                            double* gap, orc_fit* fits) {
  return reconstruct_impl(sensors, n_sensors, raw, 1, NULL, P, C, pixels, n_pixels, rgb, scale_map, margin, gap,
                          fits);
}

int orc_reconstruct_temporal(const orc_sensor* sensors, int32_t n_sensors, int32_t n_times,
                             const double* const* raw, const orc_params* P, const double* h_t,
                             const int32_t* pixels, int64_t n_pixels, double* rgb, uint8_t* scale_map,
                             double* margin, double* gap, orc_fit* fits) {
  if (n_times < 1 || n_times > ORC_MAX_TIMES || !h_t) return -8;
  for (int m = 0; m < P->n_scales; ++m)
    if (!(h_t[m] >= 0.0)) return -8;
  for (int t = 1; t < n_times; ++t) {
    const int rc = check_args(sensors, n_sensors, raw + (size_t)t * n_sensors, P, pixels, n_pixels);
    if (rc) return rc;
  }
  return reconstruct_impl(sensors, n_sensors, raw, n_times, h_t, P, NULL, pixels, n_pixels, rgb, scale_map, margin,
                          gap, fits);
}

static int reconstruct_impl(const orc_sensor* sensors, int32_t n_sensors, const double* const* raw,
                            int32_t n_times, const double* h_t, const orc_params* P, const double* Cpix,
                            const int32_t* pixels, int64_t n_pixels, double* rgb, uint8_t* scale_map,
                            double* margin, double* gap, orc_fit* fits) {
  const int rc = check_args(sensors, n_sensors, raw, P, pixels, n_pixels);
  if (rc) return rc;
  if (!rgb) return -1;
  const int M = P->order;
  const int nS = P->n_scales;
  static const int basis_size[3] = {1, 3, 6};
  sample_list list = {0, 0, 0};

  for (int64_t p = 0; p < n_pixels; ++p) {
    const int32_t u = pixels ? pixels[2 * p] : (int32_t)(p % P->out_w);
    const int32_t v = pixels ? pixels[2 * p + 1] : (int32_t)(p / P->out_w);
    double X, Y;
    affine_apply(P->out_affine, (double)u, (double)v, &X, &Y);

    for (int c = 0; c < 3; ++c) {
      const double kappa = (c == 1) ? P->green_ratio : 1.0;
      orc_fit local[ORC_MAX_SCALES][3];
      for (int m = 0; m < nS; ++m) {
        const double r = P->radii[m] * kappa;
        const double h0 = P->h[m] > 0.0 ? P->h[m] : 2.0 * P->radii[m] * P->radii[m] / 9.0;
        const double h = h0 * kappa * kappa;
        if (gather_support(sensors, n_sensors, raw, X, Y, c, r, h, Cpix ? Cpix + 3 * p : NULL, P->exhaustive,
                           n_times, h_t ? h_t[m] : 0.0, &list)) {
          free(list.v);
          return -7;
        }
        for (int o = 0; o <= M; ++o) fit_order(&list, basis_size[o], P->tau_inv, &local[m][o]);
        for (int o = M + 1; o < 3; ++o) memset(&local[m][o], 0, sizeof(orc_fit));
      }

      /* Selection: ICI at the highest order with any valid scale (R8, R9). */
      double value = NAN, mu = INFINITY, gp = INFINITY;
      int code = 0xFF;
      for (int o = M; o >= 0; --o) {
        double yh[ORC_MAX_SCALES], vr[ORC_MAX_SCALES];
        int32_t ok[ORC_MAX_SCALES];
        int any = 0;
        for (int m = 0; m < nS; ++m) {
          yh[m] = local[m][o].yhat;
          vr[m] = local[m][o].var;
          ok[m] = local[m][o].valid;
          any |= ok[m];
        }
        if (!any) continue;
        const int chosen = orc_ici_select(nS, yh, vr, ok, P->gamma, &mu, &gp);
        value = yh[chosen];
        code = (o << 4) | chosen;
        break;
      }
      rgb[3 * p + c] = value;
      if (scale_map) scale_map[3 * p + c] = (uint8_t)code;
      if (margin) margin[3 * p + c] = mu;
      if (gap) gap[3 * p + c] = gp;
      if (fits)
        for (int m = 0; m < nS; ++m)
          for (int o = 0; o < 3; ++o) fits[((p * 3 + c) * nS + m) * 3 + o] = local[m][o];
    }
  }
  free(list.v);
  return 0;
}

/* ---------------------------------------------------------------------------
 * CALPA stages (Sec. 5.4, Sec. 5.5; readings R18..R22 in lpa_oracle.h).
 * ------------------------------------------------------------------------- */

/* Stage 1: the gradient (C1) of an isotropic fit of the G channel, Sec. 5.4
 * first step with the G channel of Sec. 5.5 (R22). */
int orc_gradients(const orc_sensor* sensors, int32_t n_sensors, const double* const* raw,
                  const orc_params* P, const orc_adapt* A, const int32_t* pixels, int64_t n_pixels,
                  double* grad, int32_t* valid) {
  const int rc = check_args(sensors, n_sensors, raw, P, pixels, n_pixels);
  if (rc) return rc;
  if (!A || !grad || A->grad_order < 1 || A->grad_order > 2 || !(A->grad_radius > 0)) return -8;
  static const int basis_size[3] = {1, 3, 6};
  const double kappa = P->green_ratio;
  const double r = A->grad_radius * kappa;
  const double h0 = A->grad_h > 0.0 ? A->grad_h : 2.0 * A->grad_radius * A->grad_radius / 9.0;
  const double h = h0 * kappa * kappa;
  sample_list list = {0, 0, 0};
  for (int64_t p = 0; p < n_pixels; ++p) {
    const int32_t u = pixels ? pixels[2 * p] : (int32_t)(p % P->out_w);
    const int32_t v = pixels ? pixels[2 * p + 1] : (int32_t)(p / P->out_w);
    double X, Y;
    affine_apply(P->out_affine, (double)u, (double)v, &X, &Y);
    if (gather_support(sensors, n_sensors, raw, X, Y, 1, r, h, NULL, P->exhaustive, 1, 0.0, &list)) {
      free(list.v);
      return -7;
    }
    orc_fit fit;
    fit_order(&list, basis_size[A->grad_order], P->tau_inv, &fit);
    grad[2 * p] = fit.valid ? fit.c1x : 0.0;
    grad[2 * p + 1] = fit.valid ? fit.c1y : 0.0;
    if (valid) valid[p] = fit.valid;
  }
  free(list.v);
  return 0;
}

/* Stage 2: steering matrix of Sec. 5.4 from the gradients of the (2q+1)^2
 * output pixels around j (R20).  The singular values of the stacked gradient
 * matrix G are the square roots of the eigenvalues of G^T G; its second right
 * singular vector v is the direction of least gradient energy (along the
 * edge) and gives theta = arctan(v1 / v2).  With U_theta as printed, whose
 * second column is parallel to v, C = gamma U diag(sigma, 1/sigma) U^T
 * (R19) has eigenvalue gamma*sigma across the edge and gamma/sigma along it;
 * both are clamped (R21). */
int orc_steering(const orc_params* P, const orc_adapt* A, const double* grad_plane,
                 const int32_t* pixels, int64_t n_pixels, double* C, double* diag) {
  if (!P || !A || !grad_plane || !C) return -1;
  if (!pixels && n_pixels != (int64_t)P->out_w * P->out_h) return -5;
  if (A->grad_halfwin < 0 || !(A->max_stretch >= 1.0) || !(A->alpha >= 0.0) || !(A->lambda1 > 0.0) ||
      !(A->lambda2 >= 0.0))
    return -8;
  const int q = A->grad_halfwin;
  const double lo = 1.0 / (A->max_stretch * A->max_stretch), hi = A->max_stretch * A->max_stretch;
  for (int64_t p = 0; p < n_pixels; ++p) {
    const int32_t u = pixels ? pixels[2 * p] : (int32_t)(p % P->out_w);
    const int32_t v = pixels ? pixels[2 * p + 1] : (int32_t)(p / P->out_w);
    double txx = 0.0, txy = 0.0, tyy = 0.0;
    int count = 0;
    for (int b = -q; b <= q; ++b) {
      for (int a = -q; a <= q; ++a) {
        const int uu = u + a, vv = v + b;
        if (uu < 0 || vv < 0 || uu >= P->out_w || vv >= P->out_h) continue;
        const double gx = grad_plane[2 * ((int64_t)vv * P->out_w + uu)];
        const double gy = grad_plane[2 * ((int64_t)vv * P->out_w + uu) + 1];
        txx += gx * gx;
        txy += gx * gy;
        tyy += gy * gy;
        ++count;
      }
    }
    /* eigen-decomposition of the 2x2 symmetric G^T G */
    const double half_tr = 0.5 * (txx + tyy);
    const double disc = sqrt(0.25 * (txx - tyy) * (txx - tyy) + txy * txy);
    const double e1 = half_tr + disc;
    const double e2 = half_tr - disc > 0.0 ? half_tr - disc : 0.0;
    const double s1 = sqrt(e1), s2 = sqrt(e2);
    const double phi = 0.5 * atan2(2.0 * txy, txx - tyy); /* first right singular vector (cos, sin) */
    const double u1x = cos(phi), u1y = sin(phi);
    const double v1 = -u1y, v2 = u1x;                      /* second right singular vector */
    const double sigma = (s1 + A->lambda1) / (s2 + A->lambda1);
    const double gamma = pow((s1 * s2 + A->lambda2) / (double)count, A->alpha);
    double la = gamma * sigma, lb = gamma / sigma;
    la = la < lo ? lo : (la > hi ? hi : la);
    lb = lb < lo ? lo : (lb > hi ? hi : lb);
    /* C = la u1 u1^T + lb v v^T = lb I + (la - lb) u1 u1^T (u1 u1^T + v v^T = I) */
    C[3 * p] = lb + (la - lb) * u1x * u1x;
    C[3 * p + 1] = (la - lb) * u1x * u1y;
    C[3 * p + 2] = lb + (la - lb) * u1y * u1y;
    if (diag) {
      diag[5 * p] = s1;
      diag[5 * p + 1] = s2;
      diag[5 * p + 2] = atan(v1 / v2);
      diag[5 * p + 3] = sigma;
      diag[5 * p + 4] = gamma;
    }
  }
  return 0;
}
