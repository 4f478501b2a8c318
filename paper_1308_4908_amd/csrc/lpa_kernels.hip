// lpa_kernels.hip -- gfx950 kernels for LPA + ICI multi-sensor HDR
// reconstruction (Kronander et al., arXiv 1308.4908).
//
// Work decomposition: one workgroup per output tile, one lane per output
// pixel.  A workgroup first stages, for every sensor, the patch of samples its
// tile can reach into LDS as (radiance, inverse variance) pairs: raw DN are
// decoded there (Sec. 6 eq. Efsi, Sec. 6.1 eq. varianceestiamte, saturation
// masking) or read from a pre-pass plane.  Each lane then walks, per colour
// channel and window radius, the CFA sub-lattice points of every sensor inside
// the radius' bounding box, accumulates the weighted moments of the local
// polynomial model (Sec. 5.1, eq. wlsqe) in FP32, solves the 1x1/3x3/6x6
// normal equations in registers (LDL^T of the Jacobi-equilibrated matrix; FP64
// iterative refinement when an order-2 pivot is small) and runs ICI across radii.
//
// The normal matrix of a polynomial basis has Hankel structure: entry (i, j)
// is the weighted moment of the monomial phi_i phi_j, so an order-2 fit needs
// 15 distinct moments (not 21) and its variance matrix 15 more.
//
// Kernel families, all built on the same staging, solve and ICI code:
//   fit_kernel / fit_kernel_occ4   the isotropic fit (3- and 4-wave budgets);
//   fit_batch_kernel               its persistent form over many frames;
//   grad_kernel, steer_kernel,     adaptive anisotropic windows (Sec. 5.4,
//   fit_kernel_steer               5.5): G gradients, steering matrices, the
//                                  fit with the window d^T C d;
//   fit_kernel_stencil(_occ4)      pre-computed window weights for
//                                  translation-only rigs (scalar-load tables);
//   prepass_kernel                 raw -> FP32 or FP16 planes.
// Sensors with per-pixel calibration frames (bias, non-uniformity, readout
// variance, saturation, defects; Sec. 6) are decoded with them wherever a raw
// sample is read.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "lpa_internal.hpp"

namespace lpa {

// ---------------------------------------------------------------------------
// Polynomial basis bookkeeping.  Monomials x^p y^q with p + q <= 4 are
// numbered by degree, then by decreasing power of x.
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int midx(int p, int q) { return (p + q) * (p + q + 1) / 2 + q; }
template <int ORDER>
__host__ __device__ constexpr int n_basis() { return ORDER == 0 ? 1 : (ORDER == 1 ? 3 : 6); }
template <int ORDER>
__host__ __device__ constexpr int n_mom() { return ORDER == 0 ? 1 : (ORDER == 1 ? 6 : 15); }
// exponents of basis function i: [1, x, y, x^2, x y, y^2]
__host__ __device__ constexpr int bp(int i) { return i == 1 ? 1 : i == 3 ? 2 : i == 4 ? 1 : 0; }
__host__ __device__ constexpr int bq(int i) { return i == 2 ? 1 : i == 4 ? 1 : i == 5 ? 2 : 0; }
__host__ __device__ constexpr int aidx(int i, int j) { return midx(bp(i) + bp(j), bq(i) + bq(j)); }

// Stencil tables seen through the constant address space: uniform reads
// become scalar loads.
using ConstEntry = const __attribute__((address_space(4))) StencilEntry;
using ConstTable = const __attribute__((address_space(4))) StencilTable;

template <int ORDER, bool ICI>
struct Acc {
  float m[n_mom<ORDER>()];            // sum w * monomial
  float b[n_basis<ORDER>()];          // sum w * f * phi
  float B[ICI ? n_mom<ORDER>() : 1];  // sum K w * monomial (variance of C0)
  float f2;                           // sum w f^2 (bounds the rounding error of C0)
  // sum iv and sum iv |f| over the samples within reach (zero for tabulated
  // windows): bound the error of window weights computed from FP32 offsets
  float siv, sivf;
};

template <int ORDER, bool ICI>
__device__ __forceinline__ void acc_zero(Acc<ORDER, ICI>& a) {
#pragma unroll
  for (int k = 0; k < n_mom<ORDER>(); ++k) a.m[k] = 0.f;
#pragma unroll
  for (int k = 0; k < n_basis<ORDER>(); ++k) a.b[k] = 0.f;
#pragma unroll
  for (int k = 0; k < (ICI ? n_mom<ORDER>() : 1); ++k) a.B[k] = 0.f;
  a.f2 = 0.f;
  a.siv = 0.f;
  a.sivf = 0.f;
}

// One sample: scaled offset (dx, dy), radiance f, inverse variance iv.  The
// coordinate scale makes the Gaussian window exp2(-|d|^2); it is shifted to
// vanish at the radius and clamped to zero beyond it.  A sample at or beyond
// reach2 has exactly zero weight, so the update is skipped there: per lane,
// and for the whole wave when none of its lanes has the sample in its window.
// Returns whether the sample belongs to the support (positive weight).
// A steered window (adaptive anisotropic LPA, Sec. 5.4) replaces |d|^2 by
// the quadratic form d^T C d of the pixel's steering matrix.
struct SteerC {
  float cxx, cyy, c2xy;  // C_xx, C_yy, 2 C_xy
};

template <bool STEER>
__device__ __forceinline__ float window_r2(float dx, float dy, float x2, float y2, const SteerC& sc) {
  if constexpr (STEER) return __builtin_fmaf(sc.cxx, x2, __builtin_fmaf(sc.cyy, y2, sc.c2xy * (dx * dy)));
  else return x2 + y2;
}

// TEMP: the window is also scaled by the sample's temporal factor kt (temporal
// LPA: exp(-t^2 / h_t) of its frame), so K = K_s K_t enters w and the variance
// moments alike.
template <int ORDER, bool ICI, bool STEER, bool TEMP = false>
__device__ __forceinline__ bool acc_sample(Acc<ORDER, ICI>& a, float dx, float dy, float f, float iv,
                                           float e_edge, float reach2, const SteerC& sc, float kt = 1.f) {
  const float x2 = dx * dx, y2 = dy * dy;
  const float r2 = window_r2<STEER>(dx, dy, x2, y2, sc);
  if (r2 < reach2) {
    // K = exp2(-r2) - e_edge never exceeds 1, so clamping to [0, 1] is the
    // cut at zero (one instruction: the subtraction's clamp modifier).
    float kw = __builtin_amdgcn_fmed3f(__builtin_amdgcn_exp2f(-r2) - e_edge, 0.f, 1.f);
    // the weight-rounding sums take iv K_t: the window's slope carries K_t
    float ivt = iv;
    if constexpr (TEMP) {
      kw *= kt;
      ivt *= kt;
    }
    const float w = kw * iv;
    a.siv += ivt;
    a.sivf = __builtin_fmaf(ivt, fabsf(f), a.sivf);
    if constexpr (ORDER >= 2) {
      // Order 2: the weighted products w d^a for |a| <= 2 are the moments of
      // degree <= 2 and the basis terms of b; each moment of degree 3 and 4 is
      // one of them times dx, dy, dx^2 or dy^2 (one FMA).  B's degree <= 2
      // terms are K times the same products, its higher ones K w d^a times
      // the same factors.  Indices follow midx (degree-major, x power
      // descending): 6..9 = x^3, x^2 y, x y^2, y^3; 10..14 = x^4 .. y^4.
      const float wx = w * dx, wy = w * dy;
      const float wxx = wx * dx, wxy = wx * dy, wyy = wy * dy;
      const float p[6] = {w, wx, wy, wxx, wxy, wyy};
#pragma unroll
      for (int k = 0; k < 6; ++k) a.m[k] += p[k];
      a.m[6] = __builtin_fmaf(wxx, dx, a.m[6]);
      a.m[7] = __builtin_fmaf(wxx, dy, a.m[7]);
      a.m[8] = __builtin_fmaf(wyy, dx, a.m[8]);
      a.m[9] = __builtin_fmaf(wyy, dy, a.m[9]);
      a.m[10] = __builtin_fmaf(wxx, x2, a.m[10]);
      a.m[11] = __builtin_fmaf(wxy, x2, a.m[11]);
      a.m[12] = __builtin_fmaf(wxx, y2, a.m[12]);
      a.m[13] = __builtin_fmaf(wxy, y2, a.m[13]);
      a.m[14] = __builtin_fmaf(wyy, y2, a.m[14]);
      const float wf = w * f;
      a.b[0] += wf;
      a.f2 = __builtin_fmaf(wf, f, a.f2);
#pragma unroll
      for (int k = 1; k < 6; ++k) a.b[k] = __builtin_fmaf(f, p[k], a.b[k]);
      if constexpr (ICI) {
#pragma unroll
        for (int k = 0; k < 6; ++k) a.B[k] = __builtin_fmaf(kw, p[k], a.B[k]);
        const float kxx = kw * wxx, kxy = kw * wxy, kyy = kw * wyy;
        a.B[6] = __builtin_fmaf(kxx, dx, a.B[6]);
        a.B[7] = __builtin_fmaf(kxx, dy, a.B[7]);
        a.B[8] = __builtin_fmaf(kyy, dx, a.B[8]);
        a.B[9] = __builtin_fmaf(kyy, dy, a.B[9]);
        a.B[10] = __builtin_fmaf(kxx, x2, a.B[10]);
        a.B[11] = __builtin_fmaf(kxy, x2, a.B[11]);
        a.B[12] = __builtin_fmaf(kxx, y2, a.B[12]);
        a.B[13] = __builtin_fmaf(kxy, y2, a.B[13]);
        a.B[14] = __builtin_fmaf(kyy, y2, a.B[14]);
      }
    } else {
      // orders 0 and 1: monomials, then one FMA per moment with w, w f, w K
      float mono[n_mom<ORDER>()];
      mono[0] = 1.f;
      if constexpr (ORDER >= 1) {
        mono[1] = dx;
        mono[2] = dy;
        mono[3] = x2;
        mono[4] = dx * dy;
        mono[5] = y2;
      }
      const float wf = w * f;
      a.m[0] += w;
#pragma unroll
      for (int k = 1; k < n_mom<ORDER>(); ++k) a.m[k] = __builtin_fmaf(w, mono[k], a.m[k]);
      a.b[0] += wf;
      a.f2 = __builtin_fmaf(wf, f, a.f2);
#pragma unroll
      for (int k = 1; k < n_basis<ORDER>(); ++k) a.b[k] = __builtin_fmaf(wf, mono[k], a.b[k]);
      if constexpr (ICI) {
        const float w2 = w * kw;
        a.B[0] += w2;
#pragma unroll
        for (int k = 1; k < n_mom<ORDER>(); ++k) a.B[k] = __builtin_fmaf(w2, mono[k], a.B[k]);
      }
    }
    return w > 0.f;
  }
  return false;
}

// ---------------------------------------------------------------------------
// Register-resident solve.  LDL^T of the normal matrix A; its leading blocks
// are the factorizations of the order-1 and order-0 fits, so one
// factorization serves every order.  The pivots of the Jacobi-equilibrated
// matrix S A S (S = diag(A)^-1/2) are D_j / A_jj (the factors of S A S are
// S L S^-1 and S D S), so the equilibration need not be formed.  For order o:
// rho_o = smallest equilibrated pivot among the first n_o, valid iff rho_o >=
// tau (and the support has >= n_o samples, which the caller checks where
// rho_o does not certify it); g = A^-1 e0, C0 = g . b, var(C0) = g^T B g.
// ---------------------------------------------------------------------------
template <typename T, int ORDER>
struct Fits {
  T y[ORDER + 1];
  T v[ORDER + 1];
  T rho[ORDER + 1];
  bool ok[ORDER + 1];
  T g[ORDER + 1][n_basis<ORDER>()];  // A^-1 e0 of each order (C0 = g . b)
  // Bound on |dC0| per unit relative rounding of every moment term:
  // sum_i |g_i| sqrt(A_ii) (sqrt(F2) + sum_j sqrt(A_jj) |C_j|), F2 = sum w f^2.
  // By Cauchy-Schwarz it is at least the componentwise condition
  // |g|'|b|abs + |g|'|A|abs|C| (|.|abs: sums of absolute terms).
  T s[ORDER + 1];
};

template <typename T>
__device__ __forceinline__ T rcp_t(T x);
template <>
__device__ __forceinline__ float rcp_t<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <>
__device__ __forceinline__ double rcp_t<double>(double x) { return 1.0 / x; }

// With BOUND, the top order's s also takes the window-weight term
// edge.x * G_R * (sivf + C_R * siv), G_R = sum_i |g_i| mr^deg_i and C_R the
// same of the coefficients, mr = edge.y bounding |dx|, |dy| on the window.
template <typename T, int ORDER, bool ICI, bool BOUND = false>
__device__ __forceinline__ void solve_fits(const T* m, const T* b, const T* B, T tau, bool lower,
                                           Fits<T, ORDER>& out, T f2 = T(0), T siv = T(0), T sivf = T(0),
                                           float2 edge = float2{0.f, 0.f}) {
  constexpr int NB = n_basis<ORDER>();
  T L[NB][NB], U[NB][NB];  // U[i][k] = L[i][k] D[k]
  T D[NB], iD[NB], req[NB];
  bool dok[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    const T ajj = m[aidx(j, j)];
    dok[j] = ajj > T(0);
    T d = ajj;
#pragma unroll
    for (int k = 0; k < j; ++k) d -= U[j][k] * L[j][k];
    D[j] = d;
    iD[j] = d > T(0) ? rcp_t<T>(d) : T(0);
    req[j] = dok[j] ? d * rcp_t<T>(ajj) : T(0);  // equilibrated pivot
#pragma unroll
    for (int i = j + 1; i < NB; ++i) {
      T t = m[aidx(i, j)];
#pragma unroll
      for (int k = 0; k < j; ++k) t -= U[i][k] * L[j][k];
      U[i][j] = t;
      L[i][j] = t * iD[j];
    }
  }
  // forward substitution of e0 is shared by all orders
  T z[NB];
  z[0] = T(1);
#pragma unroll
  for (int i = 1; i < NB; ++i) {
    T t = T(0);
#pragma unroll
    for (int k = 0; k < i; ++k) t -= L[i][k] * z[k];
    z[i] = t;
  }
  // forward substitution of b and the diagonal's square roots (bound only)
  T zb[NB], sq[NB];
  if constexpr (BOUND) {
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      T t = b[i];
#pragma unroll
      for (int k = 0; k < i; ++k) t -= L[i][k] * zb[k];
      zb[i] = t;
      sq[i] = __builtin_amdgcn_sqrtf(fmaxf(m[aidx(i, i)], T(0)));
    }
  }
  T rho = T(3.0e38);
  bool diag_all = true;
#pragma unroll
  for (int o = 0; o <= ORDER; ++o) {
    constexpr int nb_tab[3] = {1, 3, 6};
    const int no = nb_tab[o];
#pragma unroll
    for (int i = (o == 0 ? 0 : nb_tab[o - 1]); i < no; ++i) {
      rho = req[i] < rho ? req[i] : rho;
      diag_all = diag_all && dok[i];
    }
    if (o < ORDER && !lower) {  // lower orders not needed (wave-uniform)
      out.y[o] = out.v[o] = out.rho[o] = out.s[o] = T(0);
      out.ok[o] = false;
#pragma unroll
      for (int i = 0; i < NB; ++i) out.g[o][i] = T(0);
      continue;
    }
    T g[NB];
#pragma unroll
    for (int i = NB - 1; i >= 0; --i) {
      if (i < no) {
        T t = z[i] * iD[i];
#pragma unroll
        for (int k = i + 1; k < NB; ++k)
          if (k < no) t -= L[k][i] * g[k];
        g[i] = t;
      } else {
        g[i] = T(0);
      }
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) out.g[o][i] = g[i];
    T y = T(0);
#pragma unroll
    for (int i = 0; i < NB; ++i)
      if (i < no) y += g[i] * b[i];
    T v = T(0);
    if constexpr (ICI) {
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        if (i < no) {
          T t = g[i] * B[aidx(i, i)];
#pragma unroll
          for (int j = i + 1; j < NB; ++j)
            if (j < no) t += T(2) * g[j] * B[aidx(i, j)];
          v += g[i] * t;
        }
      }
    }
    out.y[o] = y;
    out.v[o] = v;
    out.s[o] = T(0);
    // (the lower orders, kept for fallback, go without: a fallback output is
    // always recomputed in FP64)
    if constexpr (BOUND) if (o == ORDER) {
      T c[NB];
      T sg = T(0), scs = T(0), gr = T(0), cr = T(0);
      const T mr2 = edge.y * edge.y;
#pragma unroll
      for (int i = NB - 1; i >= 0; --i) {
        if (i < no) {
          T t = zb[i] * iD[i];
#pragma unroll
          for (int k = i + 1; k < NB; ++k)
            if (k < no) t -= L[k][i] * c[k];
          c[i] = t;
          sg = __builtin_fmaf(fabsf(g[i]), sq[i], sg);
          scs = __builtin_fmaf(fabsf(t), sq[i], scs);
          // bound of |monomial i| on the window: mr^deg (basis 0 | 1, 2 | 3, 4, 5)
          const T mono = i == 0 ? T(1) : (i < 3 ? edge.y : mr2);
          gr = __builtin_fmaf(fabsf(g[i]), mono, gr);
          cr = __builtin_fmaf(fabsf(t), mono, cr);
        } else {
          c[i] = T(0);
        }
      }
      out.s[o] = __builtin_fmaf(edge.x * gr, __builtin_fmaf(cr, siv, sivf),
                                sg * (__builtin_amdgcn_sqrtf(fmaxf(f2, T(0))) + scs));
    }
    out.rho[o] = (diag_all && rho > T(0)) ? rho : T(0);
    // Provisional: the caller also requires >= no samples where rho alone
    // does not certify it.
    out.ok[o] = diag_all && (rho >= tau);
  }
}

// ---------------------------------------------------------------------------
// FP64 moments and solve.  In HDR windows C0 is often a small difference of
// large terms (a dark pixel beside a bright edge, an exactly determined fit),
// and rounding each FP32 product and partial sum of the moments on its own
// leaves A and b mutually inconsistent by ~u relative, which that cancellation
// multiplies.  Rounding only the inputs of every moment -- offsets, window
// weight, inverse variance, radiance -- does far less harm: it is the exact fit
// of a slightly moved sample set.  The FP64 pass of ill-conditioned fits
// (validity, and the values and variances the ICI steps compare) therefore
// keeps the main pass's FP32 offsets and weights and forms products and sums
// in FP64; output values that need more are refitted from the raw frame
// (refit_kernel below).
// ---------------------------------------------------------------------------
template <int ORDER>
struct Acc64 {
  double m[n_mom<ORDER>()];
  double b[n_basis<ORDER>()];
};

template <int ORDER>
__device__ __forceinline__ void acc64_zero(Acc64<ORDER>& a) {
#pragma unroll
  for (int k = 0; k < n_mom<ORDER>(); ++k) a.m[k] = 0.0;
#pragma unroll
  for (int k = 0; k < n_basis<ORDER>(); ++k) a.b[k] = 0.0;
}

// One sample of weight w.  `hi` (wave-uniform) adds the degree-3 and 4
// moments and b's quadratic terms that an order-2 fit needs; without it only
// the order <= 1 sums are formed.
template <int ORDER, bool HAS_B = true>
__device__ __forceinline__ void acc64_sample(Acc64<ORDER>& a, float dx, float dy, float f, float w, bool hi) {
  const double wd = w, fd = f;
  a.m[0] += wd;
  if constexpr (HAS_B) a.b[0] = __builtin_fma(wd, fd, a.b[0]);
  if constexpr (ORDER >= 1) {
    const double x = dx, y = dy;
    const double wx = wd * x, wy = wd * y;
    const double wxx = wx * x, wxy = wx * y, wyy = wy * y;
    a.m[1] += wx;
    a.m[2] += wy;
    a.m[3] += wxx;
    a.m[4] += wxy;
    a.m[5] += wyy;
    if constexpr (HAS_B) {
      a.b[1] = __builtin_fma(fd, wx, a.b[1]);
      a.b[2] = __builtin_fma(fd, wy, a.b[2]);
    }
    if constexpr (ORDER >= 2) {
      if (hi) {
        const double xx = x * x, yy = y * y;
        a.m[6] = __builtin_fma(wxx, x, a.m[6]);
        a.m[7] = __builtin_fma(wxx, y, a.m[7]);
        a.m[8] = __builtin_fma(wyy, x, a.m[8]);
        a.m[9] = __builtin_fma(wyy, y, a.m[9]);
        a.m[10] = __builtin_fma(wxx, xx, a.m[10]);
        a.m[11] = __builtin_fma(wxy, xx, a.m[11]);
        a.m[12] = __builtin_fma(wxx, yy, a.m[12]);
        a.m[13] = __builtin_fma(wxy, yy, a.m[13]);
        a.m[14] = __builtin_fma(wyy, yy, a.m[14]);
        if constexpr (HAS_B) {
          a.b[3] = __builtin_fma(fd, wxx, a.b[3]);
          a.b[4] = __builtin_fma(fd, wxy, a.b[4]);
          a.b[5] = __builtin_fma(fd, wyy, a.b[5]);
        }
      }
    }
  }
}

template <int ORDER>
struct Fit64 {
  double y[ORDER + 1], rho[ORDER + 1];
  double g[ORDER + 1][n_basis<ORDER>()];  // A_o^-1 e0 of the orders solved
};

// Fits of orders 0..TOP (TOP <= ORDER) from FP64 moments: one LDL^T of the
// order-TOP normal matrix (its leading blocks are the lower orders'), the
// equilibrated pivots rho_o (0 unless every diagonal entry is positive) and,
// for the orders `want` marks, g = A_o^-1 e0 and (with HAS_B) C0 = g . b.
// Only L and z / D are kept, to hold down the registers of this rarely taken
// path.
template <int ORDER, int TOP, bool HAS_B>
__device__ __forceinline__ void solve64(const Acc64<ORDER>& a, const bool* want, Fit64<ORDER>& out) {
  constexpr int NB = n_basis<TOP>();
  constexpr int nb_tab[3] = {1, 3, 6};
  double L[NB][NB], D[NB];
  double rho = 1e300;
  bool diag = true;
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    const double ajj = a.m[aidx(j, j)];
    diag = diag && ajj > 0.0;
    double d = ajj;
#pragma unroll
    for (int k = 0; k < j; ++k) d -= L[j][k] * L[j][k] * D[k];
    D[j] = d;
    const double req = ajj > 0.0 ? d / ajj : 0.0;
    rho = req < rho ? req : rho;
    if (j + 1 < NB) {
      const double id = d > 0.0 ? 1.0 / d : 0.0;
#pragma unroll
      for (int i = j + 1; i < NB; ++i) {
        double t = a.m[aidx(i, j)];
#pragma unroll
        for (int k = 0; k < j; ++k) t -= L[i][k] * L[j][k] * D[k];
        L[i][j] = t * id;
      }
    }
#pragma unroll
    for (int o = 0; o <= TOP; ++o)
      if (j == nb_tab[o] - 1) out.rho[o] = (diag && rho > 0.0) ? rho : 0.0;
  }
  // forward substitution of e0 (shared by every order), then z_i / D_i
  double z[NB];
  z[0] = 1.0;
#pragma unroll
  for (int i = 1; i < NB; ++i) {
    double t = 0.0;
#pragma unroll
    for (int k = 0; k < i; ++k) t -= L[i][k] * z[k];
    z[i] = t;
  }
#pragma unroll
  for (int i = 0; i < NB; ++i) z[i] = D[i] > 0.0 ? z[i] / D[i] : 0.0;
#pragma unroll
  for (int o = 0; o <= ORDER; ++o) {
    out.y[o] = 0.0;
#pragma unroll
    for (int i = 0; i < n_basis<ORDER>(); ++i) out.g[o][i] = 0.0;
  }
#pragma unroll
  for (int o = 0; o <= TOP; ++o) {
    if (!want[o]) continue;
    const int no = nb_tab[o];
    double y = 0.0;
#pragma unroll
    for (int i = NB - 1; i >= 0; --i) {
      if (i < no) {
        double t = z[i];
#pragma unroll
        for (int k = i + 1; k < NB; ++k)
          if (k < no) t -= L[k][i] * out.g[o][k];
        out.g[o][i] = t;
        if constexpr (HAS_B) y = __builtin_fma(t, a.b[i], y);
      }
    }
    out.y[o] = y;
  }
#pragma unroll
  for (int o = TOP + 1; o <= ORDER; ++o) out.rho[o] = 0.0;
}

// ICI running state of one order (reading: Goldenshluger-Nemirovski rule).
struct IciState {
  float lo, hi, y, sd;
  float risk;  // chosen fit: rounding bound of C0 over max(|C0|, value floor)
               // (+inf for fits whose FP32 value carries no bound)
  int chosen;
  bool stopped, any;
};

__device__ __forceinline__ void ici_init(IciState& st) {
  st.lo = -__builtin_inff();
  st.hi = __builtin_inff();
  st.y = __builtin_nanf("");
  st.sd = __builtin_nanf("");
  st.risk = 0.f;
  st.chosen = -1;
  st.stopped = false;
  st.any = false;
}

__device__ __forceinline__ void ici_step(IciState& st, bool ok, float y, float v, float gamma, int m,
                                         float risk) {
  if (!ok) return;
  st.any = true;
  if (st.stopped) return;
  const float sd = __builtin_amdgcn_sqrtf(fmaxf(v, 0.f));
  st.lo = fmaxf(st.lo, y - gamma * sd);
  st.hi = fminf(st.hi, y + gamma * sd);
  if (st.lo <= st.hi) {
    st.chosen = m;
    st.y = y;
    st.sd = sd;
    st.risk = risk;
  } else {
    st.stopped = true;
  }
}

// ---------------------------------------------------------------------------
// Sample decode (Sec. 6 eq. Efsi, Sec. 6.1 eq. varianceestiamte): radiance
// f = (y - b) / (g n), variance (g (y - b)_+ + Var r) / (g n)^2; masked
// (y >= saturation or outside the sensor) -> (0, 0).
// ---------------------------------------------------------------------------
__device__ __forceinline__ float2 decode_dn(const SensorK& S, float y) {
  if (!(y < S.sat)) return make_float2(0.f, 0.f);
  const float yb = y - S.black;
  const float var = __builtin_fmaf(S.gain, fmaxf(yb, 0.f), S.read_var) * (S.inv_ge * S.inv_ge);
  return make_float2(yb * S.inv_ge, __builtin_amdgcn_rcpf(var));
}

// The same with the pixel's calibration frames c = (b_i, a_i, Var[r_i],
// saturation_i) (Sec. 6 eq. Efsi and varianceestiamte with a_i and the bias
// and saturation frames): scale 1 / (g n a_i).
__device__ __forceinline__ float2 decode_dn_cal(const SensorK& S, float y, float4 c) {
  if (!(y < c.w)) return make_float2(0.f, 0.f);
  const float yb = y - c.x;
  const float sc = S.inv_ge * __builtin_amdgcn_rcpf(c.y);
  const float var = __builtin_fmaf(S.gain, fmaxf(yb, 0.f), c.z) * (sc * sc);
  return make_float2(yb * sc, __builtin_amdgcn_rcpf(var));
}

// FP16 planes hold v = (y - 2^(bits-1)) 2^-bits (+Inf where masked): raw
// values of up to 12 bits come back exactly, y = v 2^bits + 2^(bits-1), so
// the decode then equals decode_dn's.  Masking was decided on the raw value.
__device__ __forceinline__ float2 decode_f16(const SensorK& S, __half h) {
  const float v = __half2float(h);
  if (__builtin_isinf(v)) return make_float2(0.f, 0.f);
  const float yb = __builtin_fmaf(v, S.norm_decode, S.norm_offset) - S.black;
  const float var = __builtin_fmaf(S.gain, fmaxf(yb, 0.f), S.read_var) * (S.inv_ge * S.inv_ge);
  return make_float2(yb * S.inv_ge, __builtin_amdgcn_rcpf(var));
}

template <int SRC>
__device__ __forceinline__ float2 load_sample(const SensorK& S, int x, int y) {
  if (x < 0 || y < 0 || x >= S.width || y >= S.height) return make_float2(0.f, 0.f);
  const char* row = static_cast<const char*>(S.src) + (int64_t)y * S.pitch;
  if constexpr (SRC == SRC_RAW_U16 || SRC == SRC_RAW_F32) {
    const float dn = SRC == SRC_RAW_U16 ? (float)reinterpret_cast<const uint16_t*>(row)[x]
                                       : reinterpret_cast<const float*>(row)[x];
    if (S.calib) return decode_dn_cal(S, dn, S.calib[(int64_t)y * S.width + x]);
    return decode_dn(S, dn);
  } else if constexpr (SRC == SRC_PLANE_F32) {
    return reinterpret_cast<const float2*>(row)[x];
  } else {
    const __half h = reinterpret_cast<const __half*>(row)[x];
    if (S.calib) {
      // as decode_f16, with the pixel's bias, scale and readout variance
      const float v = __half2float(h);
      if (__builtin_isinf(v)) return make_float2(0.f, 0.f);
      const float4 c = S.calib[(int64_t)y * S.width + x];
      const float yb = __builtin_fmaf(v, S.norm_decode, S.norm_offset) - c.x;
      const float sc = S.inv_ge * __builtin_amdgcn_rcpf(c.y);
      const float var = __builtin_fmaf(S.gain, fmaxf(yb, 0.f), c.z) * (sc * sc);
      return make_float2(yb * sc, __builtin_amdgcn_rcpf(var));
    }
    return decode_f16(S, h);
  }
}

// Region of sensor s staged for the tile at output origin (u0, v0).
struct Region {
  int x0, y0, w, h;
};

// FULL_PITCH: rows are reg_w samples apart in every tile (pre-computed-weight
// tables hold LDS offsets l * reg_w + k).
template <bool FULL_PITCH = false>
__device__ __forceinline__ Region tile_region(const LaunchK& K, const SensorK& S, int u0, int v0) {
  double mnx = 1e300, mny = 1e300, mxx = -1e300, mxy = -1e300;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const double u = u0 + ((c & 1) ? K.tile_w - 1 : 0);
    const double v = v0 + ((c & 2) ? K.tile_h - 1 : 0);
    const double X = K.out_affine[0] * u + K.out_affine[1] * v + K.out_affine[2];
    const double Y = K.out_affine[3] * u + K.out_affine[4] * v + K.out_affine[5];
    const double px = S.inv[0] * X + S.inv[1] * Y + S.inv[2];
    const double py = S.inv[3] * X + S.inv[4] * Y + S.inv[5];
    mnx = fmin(mnx, px);
    mxx = fmax(mxx, px);
    mny = fmin(mny, py);
    mxy = fmax(mxy, py);
  }
  Region r;
  r.x0 = (int)floor(mnx - S.wmax[0]) - 1;
  r.y0 = (int)floor(mny - S.wmax[1]) - 1;
  r.w = FULL_PITCH ? S.reg_w : min((int)ceil(mxx + S.wmax[0]) + 3 - r.x0 + 1, S.reg_w);
  r.h = min((int)ceil(mxy + S.wmax[1]) + 3 - r.y0 + 1, S.reg_h);
  return r;
}

template <int SRC, bool FULL_PITCH = false>
__device__ __forceinline__ void stage_tile(const LaunchK& K, int u0, int v0, float2* lds, Region* regs,
                                           int tid, int nthreads) {
  for (int s = 0; s < K.n_sensors; ++s) {
    const SensorK& S = K.s[s];
    const Region r = tile_region<FULL_PITCH>(K, S, u0, v0);
    regs[s] = r;
    float2* dst = lds + S.lds_off;
    const int total = r.w * r.h;
    for (int e = tid; e < total; e += nthreads) {
      const int row = e / r.w;
      const int col = e - row * r.w;
      dst[e] = load_sample<SRC>(S, r.x0 + col, r.y0 + row);
    }
  }
}

// Raw form of the staging (16-bit raw frames without calibration frames):
// each sample stays a 16-bit DN in LDS, a quarter of the decoded float2, and
// is decoded where a walk reads it.  Samples outside the sensor are staged as
// 0xFFFF, which no sensor's saturation (at most 65535 DN for 16-bit data)
// admits: they decode as masked, as load_sample makes them.
__device__ __forceinline__ void stage_tile_raw16(const LaunchK& K, int u0, int v0, uint16_t* lds16, Region* regs,
                                                 int tid, int nthreads) {
  for (int s = 0; s < K.n_sensors; ++s) {
    const SensorK& S = K.s[s];
    const Region r = tile_region(K, S, u0, v0);
    regs[s] = r;
    uint16_t* dst = lds16 + S.lds_off;
    const int total = r.w * r.h;
    for (int e = tid; e < total; e += nthreads) {
      const int row = e / r.w;
      const int col = e - row * r.w;
      const int x = r.x0 + col, y = r.y0 + row;
      uint16_t v = 0xFFFFu;
      if (x >= 0 && y >= 0 && x < S.width && y < S.height)
        v = reinterpret_cast<const uint16_t*>(static_cast<const char*>(S.src) + (int64_t)y * S.pitch)[x];
      dst[e] = v;
    }
  }
}

// ---------------------------------------------------------------------------
// Per-pixel fit of one tile.  All loop bounds are uniform across the wave.
// ---------------------------------------------------------------------------

// Fits whose equilibrated pivot is below tau_fp64 (ill-conditioned) get their
// variance recomputed from the samples as sum_k (g . phi_k)^2 K_k w_k (all
// terms positive) instead of the moment form g^T B g.  Above it both forms
// carry ~1e-4 relative error or less in FP32; below it the moment form's
// cancellation grows quickly.
//
// An FP32 pivot carries the moments' rounding amplified by the inverse of the
// pivots before it.  While every pivot of a fit stays above kPivotCertifiesN
// that error is far below tau and below the pivot itself, so the FP32
// factorization decides the fit, and its matrix being regular certifies
// N >= n_o.  A fit with a smaller pivot is decided by the second pass: its
// samples are counted and its normal matrix re-accumulated in FP64.
constexpr float kPivotCertifiesN = 1e-3f;

// Visits an nx x ny box of sub-lattice points in blocks of kBlk x kBlk: the
// block body is unrolled behind uniform guards, so offsets advance by uniform
// steps, LDS reads use immediate offsets, and every box size runs the same
// code (separately inlined walks per size would make the compiler copy each
// accumulator where they merge).
constexpr int kBlk = 5;

template <typename T, class Fn>
__device__ __forceinline__ void walk_box(const T* p0, int row_step, int nx, int ny, float c0x, float c0y,
                                         float sax, float say, float sbx, float sby, Fn& fn) {
  for (int jb = 0; jb < ny; jb += kBlk) {
    for (int ib = 0; ib < nx; ib += kBlk) {
      const int mx = nx - ib, my = ny - jb;
      const T* pb = p0 + jb * row_step + 2 * ib;
      float rx = __builtin_fmaf((float)ib, sax, __builtin_fmaf((float)jb, sbx, c0x));
      float ry = __builtin_fmaf((float)ib, say, __builtin_fmaf((float)jb, sby, c0y));
#pragma unroll
      for (int jj = 0; jj < kBlk; ++jj) {
        if (jj < my) {
          const T* prow = pb + jj * row_step;
          float dx = rx, dy = ry;
#pragma unroll
          for (int ii = 0; ii < kBlk; ++ii) {
            if (ii < mx) {
              fn(dx, dy, prow[2 * ii]);
              dx += sax;
              dy += say;
            }
          }
          rx += sbx;
          ry += sby;
        }
      }
    }
  }
}

// Wave-wide bounds on the entries of C^-1 over the wave's steered windows
// (|.| for the off-diagonal one).  The ellipse d^T C d < r^2 spans
// r sqrt(a^T C^-1 a) along a direction a, and a^T C^-1 a <= ax^2 pxx +
// 2 |ax ay| pxy + ay^2 pyy for every lane of the wave.
struct SteerBox {
  float pxx, pyy, pxy;
};

__device__ __forceinline__ float wave_max(float x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x = fmaxf(x, __shfl_xor(x, d, 64));
  return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, x)));
}

// Calls fn(dx, dy, f, iv, s) for every CFA sample of channel c inside the box of
// radius index m around (Xj, Yj), over all sensors (scaled offsets).  The
// box holds the disk of the radius; for steered windows, the wave's ellipses
// (half-widths from SteerBox, at most the box of the largest stretch, which
// the staged tile region covers).
template <bool STEER, bool RAW16 = false, class Fn>
__device__ __forceinline__ void walk_support(const LaunchK& K, const float2* lds, const Region* regs,
                                             double Xj, double Yj, int c, int cls, int m, const SteerBox& sb,
                                             Fn&& fn) {
  const ScaleK& SC = K.sc[m];
  const double rad = SC.box_radius[cls];
  const float cs = SC.coord_scale[cls];
  for (int s = 0; s < K.n_sensors; ++s) {
    const SensorK& S = K.s[s];
    const Region R = regs[s];
    // lane position on the sensor and the box half-widths of this radius
    const double px = S.inv[0] * Xj + S.inv[1] * Yj + S.inv[2];
    const double py = S.inv[3] * Xj + S.inv[4] * Yj + S.inv[5];
    double wx = rad * S.rownorm[0];
    double wy = rad * S.rownorm[1];
    int nx = S.nbox[cls][m][0];
    int ny = S.nbox[cls][m][1];
    if constexpr (STEER) {
      const float ax = (float)S.inv[0], ay = (float)S.inv[1], bx = (float)S.inv[3], by = (float)S.inv[4];
      const float qx = ax * ax * sb.pxx + 2.f * fabsf(ax * ay) * sb.pxy + ay * ay * sb.pyy;
      const float qy = bx * bx * sb.pxx + 2.f * fabsf(bx * by) * sb.pxy + by * by * sb.pyy;
      const float r = (float)SC.radius[cls] * 1.001f;  // margin over rounding of the bound
      wx = fmin((double)(r * __builtin_amdgcn_sqrtf(qx)), wx);
      wy = fmin((double)(r * __builtin_amdgcn_sqrtf(qy)), wy);
      nx = __builtin_amdgcn_readfirstlane(min(nx, max(1, (int)ceil(wx - 1e-9))));
      ny = __builtin_amdgcn_readfirstlane(min(ny, max(1, (int)ceil(wy - 1e-9))));
    }
    // step between sub-lattice points (+2 px in x or y), scaled
    const float sax = (float)(2.0 * S.fwd[0] * cs), say = (float)(2.0 * S.fwd[3] * cs);
    const float sbx = (float)(2.0 * S.fwd[1] * cs), sby = (float)(2.0 * S.fwd[4] * cs);
    const int row_step = 2 * R.w;
    const int nsub = S.sub_n[c];
    for (int q = 0; q < nsub; ++q) {
      const int ox = S.sub_ox[c][q], oy = S.sub_oy[c][q];
      // first sub-lattice point with |x - px| < wx (same for y)
      const int xb = ox + 2 * (int)ceil((px - wx - ox) * 0.5);
      const int yb = oy + 2 * (int)ceil((py - wy - oy) * 0.5);
      // offset of that point from the output position, formed in FP64
      const double Xb = S.fwd[0] * xb + S.fwd[1] * yb + S.fwd[2];
      const double Yb = S.fwd[3] * xb + S.fwd[4] * yb + S.fwd[5];
      const float c0x = (float)((Xb - Xj) * cs);
      const float c0y = (float)((Yb - Yj) * cs);
      // row index times pitch: both are below 2^24 (the box lies inside the
      // staged region), so the full-rate 24-bit multiply is exact
      const int at = S.lds_off + __mul24(yb - R.y0, R.w) + (xb - R.x0);
      if constexpr (RAW16) {
        const uint16_t* p0 = reinterpret_cast<const uint16_t*>(lds) + at;
        auto fs = [&](float dx, float dy, uint16_t dn) {
          const float2 d = decode_dn(S, (float)dn);
          fn(dx, dy, d.x, d.y, s);
        };
        walk_box(p0, row_step, nx, ny, c0x, c0y, sax, say, sbx, sby, fs);
      } else {
        const float2* p0 = lds + at;
        auto fs = [&](float dx, float dy, float2 sm) { fn(dx, dy, sm.x, sm.y, s); };
        walk_box(p0, row_step, nx, ny, c0x, c0y, sax, say, sbx, sby, fs);
      }
    }
  }
}

// Workgroups are dispatched to the 8 XCDs round-robin (workgroup i runs on
// XCD i mod 8), each with its own L2.  Giving XCD x a contiguous range of
// tiles keeps the halo a tile shares with its neighbours in that XCD's L2
// instead of fetching it from HBM once per XCD.  A bijection on [0, n).
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_tile(int i, int n) {
  const int q = n / kXcds, r = n - q * kXcds;
  const int x = i % kXcds, j = i / kXcds;
  return x * q + (x < r ? x : r) + j;
}

// ---------------------------------------------------------------------------
// FP64 refit from the raw frame.  Outputs whose FP32 value could be off by
// more than the target are recomputed as the model defines them, in FP64
// throughout: each raw sample is re-read from the frame and decoded (Sec. 6
// eq. Efsi, Sec. 6.1 eq. varianceestiamte, with the pixel's calibration
// frames), placed by the FP64 sensor map (Sec. 4.2), weighted by the FP64
// window of the chosen radius, and the normal equations are accumulated and
// solved in FP64.  Where C0 is a small difference of large terms, even the
// FP32 rounding of a sample's position or weight moves it by more than the
// target, so the refit keeps nothing of the FP32 pass but its decision.
// ---------------------------------------------------------------------------
// 1 / x to FP64 accuracy: the hardware reciprocal and one Newton step.
__device__ __forceinline__ double rcp64(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  return __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
}

// exp(-t) for t >= 0 in FP64 (relative error ~1e-15): with x = -t log2(e) =
// n + r, n = rint(x), |r| <= 1/2, exp(-t) = 2^n exp(r ln 2), and exp(s),
// |s| <= ln(2) / 2, from its Taylor series to degree 12 (remainder below
// 0.35^13 / 13! ~ 2e-16), evaluated by Horner's rule.
__device__ __forceinline__ double exp_neg64(double t) {
  const double x = -t * 1.4426950408889634;
  const double n = __builtin_rint(x);
  const double s = (x - n) * 0.6931471805599453;
  double p = 1.0 / 479001600.0;  // 1 / 12!
  p = __builtin_fma(p, s, 1.0 / 39916800.0);
  p = __builtin_fma(p, s, 1.0 / 3628800.0);
  p = __builtin_fma(p, s, 1.0 / 362880.0);
  p = __builtin_fma(p, s, 1.0 / 40320.0);
  p = __builtin_fma(p, s, 1.0 / 5040.0);
  p = __builtin_fma(p, s, 1.0 / 720.0);
  p = __builtin_fma(p, s, 1.0 / 120.0);
  p = __builtin_fma(p, s, 1.0 / 24.0);
  p = __builtin_fma(p, s, 1.0 / 6.0);
  p = __builtin_fma(p, s, 0.5);
  p = __builtin_fma(p, s, 1.0);
  p = __builtin_fma(p, s, 1.0);
  return n < -1060.0 ? 0.0 : __builtin_amdgcn_ldexp(p, (int)n);
}

// Radiance and inverse variance of raw value dn at sensor pixel i (row-major
// index) in FP64: f = (dn - b) / (g n a), Var f = (g max(f, 0) + Var[r] / (g n a))
// / (g n a), with the pixel's calibration frames where the sensor has them.
// Returns false where the sample is masked.
__device__ __forceinline__ bool decode64(const SensorK& S, int64_t i, double dn, double& f, double& iv) {
  double b = S.black64, rv = S.read_var64, sat = S.sat64, inv_ga = S.inv_ge64;
  if (S.calib) {
    const float4 c = S.calib[i];
    b = c.x;
    inv_ga *= rcp64((double)c.y);
    rv = c.z;
    sat = c.w;
  }
  if (!(dn < sat)) return false;
  f = (dn - b) * inv_ga;
  iv = rcp64(inv_ga * __builtin_fma(S.gain64, fmax(f, 0.0), rv * inv_ga));
  return true;
}

// One FP64 sample (unscaled offset x, y; radiance f; weight w) into the
// normal equations of every order up to ORDER.
template <int ORDER>
__device__ __forceinline__ void acc64_d(Acc64<ORDER>& a, double x, double y, double f, double w) {
  a.m[0] += w;
  a.b[0] = __builtin_fma(w, f, a.b[0]);
  if constexpr (ORDER >= 1) {
    const double wx = w * x, wy = w * y;
    const double wxx = wx * x, wxy = wx * y, wyy = wy * y;
    a.m[1] += wx;
    a.m[2] += wy;
    a.m[3] += wxx;
    a.m[4] += wxy;
    a.m[5] += wyy;
    a.b[1] = __builtin_fma(f, wx, a.b[1]);
    a.b[2] = __builtin_fma(f, wy, a.b[2]);
    if constexpr (ORDER >= 2) {
      const double xx = x * x, yy = y * y;
      a.m[6] = __builtin_fma(wxx, x, a.m[6]);
      a.m[7] = __builtin_fma(wxx, y, a.m[7]);
      a.m[8] = __builtin_fma(wyy, x, a.m[8]);
      a.m[9] = __builtin_fma(wyy, y, a.m[9]);
      a.m[10] = __builtin_fma(wxx, xx, a.m[10]);
      a.m[11] = __builtin_fma(wxy, xx, a.m[11]);
      a.m[12] = __builtin_fma(wxx, yy, a.m[12]);
      a.m[13] = __builtin_fma(wxy, yy, a.m[13]);
      a.m[14] = __builtin_fma(wyy, yy, a.m[14]);
      a.b[3] = __builtin_fma(f, wxx, a.b[3]);
      a.b[4] = __builtin_fma(f, wxy, a.b[4]);
      a.b[5] = __builtin_fma(f, wyy, a.b[5]);
    }
  }
}

// C0 of output pixel (u, v), channel c, at radius index m and order o (<=
// ORDER), in FP64 from the raw frame (its samples staged in LDS, `raw` with
// the tile's regions `regs`); steered windows read the pixel's steering
// matrix.  Every sensor's box covers the window: the disc of radius
// r' (the ellipse d^T C d < r'^2, whose half-width along a sensor axis with
// inverse-map row a is r' sqrt(a^T C^-1 a)).  One lane per output.
template <int ORDER, bool STEER, typename RawT>
__device__ double refit_one(const LaunchK& K, const RawT* raw, const Region* regs, const int* offs, int u, int v,
                            int c, int o, int m) {
  const double Xj = K.out_affine[0] * u + K.out_affine[1] * v + K.out_affine[2];
  const double Yj = K.out_affine[3] * u + K.out_affine[4] * v + K.out_affine[5];
  const int cls = (c == 1) ? 1 : 0;
  const double r = K.sc[m].radius[cls];
  const double r2 = r * r, ih = 1.0 / K.sc[m].h[cls];
  const double ee = exp_neg64(r2 * ih);
  double cxx = 1.0, cxy = 0.0, cyy = 1.0, ixx = 1.0, ixy = 0.0, iyy = 1.0;  // C and C^-1
  if constexpr (STEER) {
    const float4 q = reinterpret_cast<const float4*>(reinterpret_cast<const char*>(K.steer) +
                                                     (int64_t)v * K.steer_pitch)[u];
    cxx = q.x;
    cxy = q.y;
    cyy = q.z;
    const double id = 1.0 / (cxx * cyy - cxy * cxy);
    ixx = cyy * id;
    iyy = cxx * id;
    ixy = -cxy * id;
  }
  Acc64<ORDER> a;
  acc64_zero(a);
  for (int s = 0; s < K.n_sensors; ++s) {
    const SensorK& S = K.s[s];
    const Region R = regs[s];
    const RawT* plane = raw + offs[s];
    // the frame's temporal factor exp(-t^2 / h_t) (temporal LPA; 1 at t = 0,
    // 0 where the FP32 pass has it 0: h_t = 0)
    const double kt =
        S.time == 0 ? 1.0 : (S.kt[m] == 0.f ? 0.0 : exp_neg64((double)S.time * S.time * K.sc[m].inv_ht));
    const double px = S.inv[0] * Xj + S.inv[1] * Yj + S.inv[2];
    const double py = S.inv[3] * Xj + S.inv[4] * Yj + S.inv[5];
    const double ax = S.inv[0], ay = S.inv[1], bx = S.inv[3], by = S.inv[4];
    const double wx = r * sqrt(ax * ax * ixx + 2.0 * ax * ay * ixy + ay * ay * iyy) * (1.0 + 1e-12);
    const double wy = r * sqrt(bx * bx * ixx + 2.0 * bx * by * ixy + by * by * iyy) * (1.0 + 1e-12);
    const int nx = max(1, (int)ceil(wx - 1e-9)), ny = max(1, (int)ceil(wy - 1e-9));
    // one step along a sub-lattice row (+2 sensor px in x), in the reference
    // plane; d2 along the row is quadratic in the step index, so the window's
    // exp(-d2 / h) is a product recurrence: e_{i+1} = e_i q_i, q_{i+1} = q_i cq
    const double sx = 2.0 * S.fwd[0], sy = 2.0 * S.fwd[3];
    const double qs = cxx * sx * sx + 2.0 * cxy * sx * sy + cyy * sy * sy;  // second difference / 2
    const double cq = exp_neg64(2.0 * qs * ih);
    for (int q = 0; q < S.sub_n[c]; ++q) {
      const int ox = S.sub_ox[c][q], oy = S.sub_oy[c][q];
      const int xb = ox + 2 * (int)ceil((px - wx - ox) * 0.5);
      const int yb = oy + 2 * (int)ceil((py - wy - oy) * 0.5);
      for (int j = 0; j < ny; ++j) {
        const int y = yb + 2 * j;
        if (y < 0 || y >= S.height) continue;
        const RawT* row = plane + (y - R.y0) * R.w - R.x0;
        // the row's first point: its window exponent and the first step's factor
        const double dX0 = S.fwd[0] * xb + S.fwd[1] * y + S.fwd[2] - Xj;
        const double dY0 = S.fwd[3] * xb + S.fwd[4] * y + S.fwd[5] - Yj;
        const double d20 = cxx * dX0 * dX0 + 2.0 * cxy * dX0 * dY0 + cyy * dY0 * dY0;
        const double lin = 2.0 * (cxx * dX0 * sx + cxy * (dX0 * sy + dY0 * sx) + cyy * dY0 * sy);
        double e = exp_neg64(d20 * ih);
        double qf = exp_neg64((lin + qs) * ih);
        for (int i = 0; i < nx; ++i, e *= qf, qf *= cq) {
          const int x = xb + 2 * i;
          if (x < 0 || x >= S.width) continue;
          const double dX = S.fwd[0] * x + S.fwd[1] * y + S.fwd[2] - Xj;
          const double dY = S.fwd[3] * x + S.fwd[4] * y + S.fwd[5] - Yj;
          const double d2 = STEER ? cxx * dX * dX + 2.0 * cxy * dX * dY + cyy * dY * dY : dX * dX + dY * dY;
          if (!(d2 < r2)) continue;
          double f, iv;
          if (decode64(S, (int64_t)y * S.width + x, (double)row[x], f, iv))
            acc64_d<ORDER>(a, dX, dY, f, (e - ee) * kt * iv);
        }
      }
    }
  }
  bool want[ORDER + 1];
#pragma unroll
  for (int k = 0; k <= ORDER; ++k) want[k] = k == o;
  Fit64<ORDER> fit;
  solve64<ORDER, ORDER, true>(a, want, fit);
  double y = 0.0;
#pragma unroll
  for (int k = 0; k <= ORDER; ++k)
    if (k == o) y = fit.y[k];
  return y;
}

// The refit of one tile: its marked outputs are gathered in LDS ordered by
// (channel, radius) -- a counting sort, so the lanes of a wave mostly walk
// boxes of one shape -- then each lane of the workgroup takes one.
constexpr int kRefitClasses = 3 * kMaxScales;
constexpr int kRefitThreads = 256;  // one workgroup per output block
constexpr int kRefitMaxOut = 32 * 32 * 3;

// Sensor footprint staged for the output block at (u0, v0) of cw x ch
// pixels: the block corners' sensor positions widened by the largest box
// half-width and a margin (the host bounds its size by the same rule).
__device__ __forceinline__ Region block_region(const LaunchK& K, const SensorK& S, int u0, int v0, int cw, int ch) {
  double mnx = 1e300, mny = 1e300, mxx = -1e300, mxy = -1e300;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const double u = u0 + ((c & 1) ? cw - 1 : 0);
    const double v = v0 + ((c & 2) ? ch - 1 : 0);
    const double X = K.out_affine[0] * u + K.out_affine[1] * v + K.out_affine[2];
    const double Y = K.out_affine[3] * u + K.out_affine[4] * v + K.out_affine[5];
    const double px = S.inv[0] * X + S.inv[1] * Y + S.inv[2];
    const double py = S.inv[3] * X + S.inv[4] * Y + S.inv[5];
    mnx = fmin(mnx, px);
    mxx = fmax(mxx, px);
    mny = fmin(mny, py);
    mxy = fmax(mxy, py);
  }
  Region r;
  r.x0 = (int)floor(mnx - S.wmax[0]) - 1;
  r.y0 = (int)floor(mny - S.wmax[1]) - 1;
  r.w = (int)ceil(mxx + S.wmax[0]) + 3 - r.x0 + 1;
  r.h = (int)ceil(mxy + S.wmax[1]) + 3 - r.y0 + 1;
  return r;
}

// The FP64 refit of the marked outputs of one output block (K.refit_bw x
// K.refit_bh pixels, row-major block number b): the marks are gathered in LDS
// ordered by (channel, radius) -- a counting sort, so the lanes of a wave
// mostly walk boxes of one shape -- the block's raw samples are staged, and
// each lane refits one output.  Every output is computed by one lane from
// the same samples in the same order whatever the block, tile or batch.
// CLOSE: end with a workgroup barrier.  Without one, waves without an output
// end early and free their registers for other workgroups' waves; the batch
// kernel keeps it (without it the compiler's schedule of the three inlined
// orders spills 224 bytes per lane at its 4-wave budget instead of 136).
template <int ORDER, bool STEER, typename RawT, bool CLOSE = false>
__device__ __forceinline__ void refit_block(const LaunchK& K, int b, uint16_t* list, int* count, RawT* raw,
                                            Region* regs, int* offs) {
  const int bx = (K.out_w + K.refit_bw - 1) / K.refit_bw;
  const int u0 = (b % bx) * K.refit_bw, v0 = (b / bx) * K.refit_bh;
  const int cw = min(K.refit_bw, K.out_w - u0), ch = min(K.refit_bh, K.out_h - v0);
  const int n_out = cw * ch * 3;
  const int tid = threadIdx.x;
  for (int k = tid; k <= kRefitClasses; k += kRefitThreads) count[k] = 0;
  __syncthreads();
  constexpr int kCodes = kRefitMaxOut / kRefitThreads;
  uint8_t codes[kCodes];
#pragma unroll
  for (int k = 0; k < kCodes; ++k) {
    const int t = tid + k * kRefitThreads;
    const int p = t / 3, c = t - 3 * p;
    codes[k] = t < n_out ? K.refit_map[(int64_t)(v0 + p / cw) * K.refit_pitch + 3 * (u0 + p % cw) + c] : 0;
    if (codes[k] & 0x80) atomicAdd(&count[1 + c * kMaxScales + (codes[k] & 7)], 1);
  }
  __syncthreads();
  if (tid == 0)
    for (int k = 1; k <= kRefitClasses; ++k) count[k] += count[k - 1];  // count[k]: start of class k
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kCodes; ++k) {
    const int t = tid + k * kRefitThreads;
    if (codes[k] & 0x80) list[atomicAdd(&count[(t % 3) * kMaxScales + (codes[k] & 7)], 1)] = (uint16_t)t;
  }
  __syncthreads();
  const int n = count[kRefitClasses - 1];
  if (n == 0) return;  // workgroup-uniform
  if (tid == 0) {
    int off = 0;
    for (int s = 0; s < K.n_sensors; ++s) {
      const Region r = block_region(K, K.s[s], u0, v0, cw, ch);
      regs[s] = r;
      offs[s] = off;
      off += r.w * r.h;
    }
  }
  __syncthreads();
  // the block's raw samples, kStageRun per lane at a time so that their loads
  // are in flight together
  constexpr int kStageRun = 8;
  for (int s = 0; s < K.n_sensors; ++s) {
    const SensorK& S = K.s[s];
    const Region r = regs[s];
    RawT* dst = raw + offs[s];
    const int total = r.w * r.h;
    for (int e0 = tid; e0 < total; e0 += kStageRun * kRefitThreads) {
      RawT val[kStageRun];
#pragma unroll
      for (int k = 0; k < kStageRun; ++k) {
        const int e = e0 + k * kRefitThreads;
        const int row = e / r.w, col = e - row * r.w;
        const int x = r.x0 + col, y = r.y0 + row;
        val[k] = RawT(0);
        if (e < total && x >= 0 && y >= 0 && x < S.width && y < S.height)
          val[k] = reinterpret_cast<const RawT*>(static_cast<const char*>(S.raw) + (int64_t)y * S.raw_pitch)[x];
      }
#pragma unroll
      for (int k = 0; k < kStageRun; ++k)
        if (e0 + k * kRefitThreads < total) dst[e0 + k * kRefitThreads] = val[k];
    }
  }
  __syncthreads();
  for (int i = tid; i < n; i += kRefitThreads) {
    const int t = list[i];
    const int p = t / 3, c = t - 3 * p;
    const int u = u0 + p % cw, v = v0 + p / cw;
    const int code = K.refit_map[(int64_t)v * K.refit_pitch + 3 * u + c];
    const double y = refit_one<ORDER, STEER>(K, raw, regs, offs, u, v, c, (code >> 4) & 3, code & 7);
    float* orow = reinterpret_cast<float*>(reinterpret_cast<char*>(K.rgb) + (int64_t)v * K.rgb_pitch);
    orow[3 * u + c] = (float)y;
  }
  if constexpr (CLOSE) __syncthreads();
}

// One workgroup per output block; dynamic LDS: the raw samples of the block's
// footprints (K.refit_lds elements of RawT: uint16 frames as uint16, float DN
// as float).  Compiled for 4 waves per SIMD: the FP64 walks are latency-bound,
// and the extra waves outweigh the registers spilled to reach 128 VGPRs.
template <int ORDER, bool STEER, typename RawT>
__global__ void __launch_bounds__(kRefitThreads) __attribute__((amdgpu_waves_per_eu(4, 8)))
refit_kernel(const LaunchK K) {
  extern __shared__ float2 lds[];
  __shared__ uint16_t list[kRefitMaxOut];
  __shared__ int count[kRefitClasses + 1];
  __shared__ Region regs[kMaxSensors];
  __shared__ int offs[kMaxSensors];
  // neighbouring blocks on one XCD share their halos in its L2
  refit_block<ORDER, STEER, RawT>(K, xcd_tile(blockIdx.x, gridDim.x), list, count, reinterpret_cast<RawT*>(lds), regs,
                                  offs);
}

// Batch form: the batch's blocks, frame after frame, are numbered 0, 1, ...
// (frames without refits have no blocks); one workgroup per block, as in
// refit_kernel.  (A persistent loop over blocks costs the order-2 refit
// about 85 more VGPRs, and with them half its occupancy.)
template <typename RawT>
__device__ __forceinline__ void refit_batch_frame(const LaunchK& K, int b, uint16_t* list, int* count, RawT* raw,
                                                  Region* regs, int* offs) {
  switch (K.order) {
    case 0: refit_block<0, false, RawT, true>(K, b, list, count, raw, regs, offs); break;
    case 1: refit_block<1, false, RawT, true>(K, b, list, count, raw, regs, offs); break;
    default: refit_block<2, false, RawT, true>(K, b, list, count, raw, regs, offs); break;
  }
}

// (all frames of a batch share the raw element type RawT; 4 waves per SIMD,
// as refit_kernel.)  Workgroup i runs
// on XCD x = i mod 8 (round-robin dispatch) as that XCD's j = i / 8-th
// workgroup.  Each XCD takes the x-th eighth of every frame's blocks, frame
// after frame: neighbouring blocks share their halos in its L2, and every XCD
// gets a share of every frame (frames differ widely in how many outputs they
// mark; contiguous ranges of the batch would leave some XCDs idle).  The grid
// is 8 x the largest per-XCD block count; workgroups past their XCD's count
// return at once.
template <typename RawT>
__global__ void __launch_bounds__(kRefitThreads) __attribute__((amdgpu_waves_per_eu(4, 8)))
refit_batch_kernel(const BatchHeader* __restrict__ hdr,
                                                                    const LaunchK* __restrict__ frames,
                                                                    const int64_t* __restrict__ first_tile) {
  (void)first_tile;
  extern __shared__ float2 lds[];
  __shared__ uint16_t list[kRefitMaxOut];
  __shared__ int count[kRefitClasses + 1];
  __shared__ Region regs[kMaxSensors];
  __shared__ int offs[kMaxSensors];
  const int n_frames = hdr->n_frames;
  const int x = (int)(blockIdx.x % kXcds);
  const int64_t j = blockIdx.x / kXcds;
  int64_t base = 0, lo = 0;
  int f = 0;
  for (; f < n_frames; ++f) {
    const LaunchK& K = frames[f];
    if (!K.refit_map) continue;
    const int64_t nb = (int64_t)((K.out_w + K.refit_bw - 1) / K.refit_bw) * ((K.out_h + K.refit_bh - 1) / K.refit_bh);
    const int64_t a = nb * x / kXcds, b = nb * (x + 1) / kXcds;  // this XCD's slice
    if (j < base + (b - a)) {
      lo = a;
      break;
    }
    base += b - a;
  }
  if (f >= n_frames) return;
  refit_batch_frame<RawT>(frames[f], (int)(lo + (j - base)), list, count, reinterpret_cast<RawT*>(lds), regs, offs);
}

// Pre-computed window weights: one tabulated sample of a stencil.  The entry
// holds K * monomial for every Hankel moment, so A, b and B take one FMA per
// moment each (w = K iv, w f and K w are formed once per sample).  Returns
// whether the sample belongs to the support (positive inverse variance).
template <int ORDER, bool ICI>
__device__ __forceinline__ bool acc_entry(Acc<ORDER, ICI>& a, const ConstEntry& e, float f, float iv) {
  const float wf = f * iv;
  a.f2 = __builtin_fmaf(e.a[0] * wf, f, a.f2);
#pragma unroll
  for (int k = 0; k < n_mom<ORDER>(); ++k) a.m[k] = __builtin_fmaf(e.a[k], iv, a.m[k]);
#pragma unroll
  for (int k = 0; k < n_basis<ORDER>(); ++k) a.b[k] = __builtin_fmaf(e.a[k], wf, a.b[k]);
  if constexpr (ICI) {
    const float wk = e.a[0] * iv;  // a[0] = K
#pragma unroll
    for (int k = 0; k < n_mom<ORDER>(); ++k) a.B[k] = __builtin_fmaf(e.a[k], wk, a.B[k]);
  }
  return iv > 0.f;
}

// Calls fn(entry, f, iv) for every tabulated sample of channel c, radius index
// m, for the wave's output-pixel parity `par` (uniform: a 256-lane tile puts
// one parity class in each wave).  Entries are read through the constant
// address space with uniform addresses: scalar loads, no vector registers.
template <class Fn>
__device__ __forceinline__ void walk_stencil(const LaunchK& K, const float2* lds, const Region* regs, int u, int v,
                                             int c, int par, int m, Fn&& fn) {
  // a C-style cast is the address-space cast (generic -> constant)
  const ConstTable* T = (const ConstTable*)K.stencil;
  const ConstEntry* E = (const ConstEntry*)((const __attribute__((address_space(4))) char*)T +
                                            StencilTable::entries_offset());
  for (int s = 0; s < K.n_sensors; ++s) {
    const int off = T->seg[c][par][m][s].off, n = T->seg[c][par][m][s].n;
    const Region R = regs[s];
    // LDS index of sensor pixel (u, v) in the staged region (row pitch reg_w;
    // it may lie outside the region, every tabulated sample lies inside it)
    const int base = K.s[s].lds_off + (v - R.y0) * K.s[s].reg_w + (u - R.x0);
    // pairs: one wait covers both entries' scalar loads, one both LDS reads
    int i = 0;
    for (; i + 1 < n; i += 2) {
      const ConstEntry& e0 = E[off + i];
      const ConstEntry& e1 = E[off + i + 1];
      const float2 f0 = lds[base + e0.delta];
      const float2 f1 = lds[base + e1.delta];
      fn(e0, f0.x, f0.y);
      fn(e1, f1.x, f1.y);
    }
    if (i < n) {
      const ConstEntry& e = E[off + i];
      const float2 fi = lds[base + e.delta];
      fn(e, fi.x, fi.y);
    }
  }
}

// cnt64 / cnt_nan count this lane's outputs marked for the FP64 refit and
// those with no valid fit.
template <int ORDER, bool ICI, bool STEER, bool STENCIL = false, bool TEMP = false, bool RAW16 = false>
__device__ __forceinline__ void fit_pixel(const LaunchK& K, const float2* lds, const Region* regs,
                                          int u, int v, bool active, int& cnt64, int& cnt_nan) {
  const double Xj = K.out_affine[0] * u + K.out_affine[1] * v + K.out_affine[2];
  const double Yj = K.out_affine[3] * u + K.out_affine[4] * v + K.out_affine[5];
  SteerC sc = {1.f, 1.f, 0.f};  // lanes outside the grid keep the isotropic window (inside the box)
  SteerBox sb = {0.f, 0.f, 0.f};
  // the window's extent along x and y over its isotropic radius: on the
  // ellipse d^T C d < r^2, |d_x| <= r sqrt((C^-1)_xx)
  float stretch = 1.f;
  if constexpr (STEER) {
    float pxx = 0.f, pyy = 0.f, pxy = 0.f;  // C^-1 of the active lanes
    if (active) {
      const float4 c = reinterpret_cast<const float4*>(reinterpret_cast<const char*>(K.steer) +
                                                       (int64_t)v * K.steer_pitch)[u];
      sc = {c.x, c.z, 2.f * c.y};
      const float id = 1.f / (c.x * c.z - c.y * c.y);
      pxx = c.z * id;
      pyy = c.x * id;
      pxy = fabsf(c.y * id);
      stretch = sqrtf(fmaxf(pxx, pyy));
    }
    sb = {wave_max(pxx), wave_max(pyy), wave_max(pxy)};
  }
  const int par = __builtin_amdgcn_readfirstlane((u & 1) + 2 * (v & 1));
  for (int c = 0; c < 3; ++c) {
    const int cls = (c == 1) ? 1 : 0;
    IciState st[ORDER + 1];
#pragma unroll
    for (int o = 0; o <= ORDER; ++o) ici_init(st[o]);

    for (int m = 0; m < K.n_scales; ++m) {
      const float eedge = K.sc[m].e_edge[cls];
      const float reach2 = K.sc[m].reach2[cls];
      Acc<ORDER, ICI> a;
      acc_zero(a);
      // At the first (smallest) radius the support is often smaller than the
      // number of unknowns; the walk counts it there, which decides those fits
      // without a second pass.  Elsewhere the count is taken only when needed.
      int n_first = -1;
      if constexpr (STENCIL) {
        if (m == 0) {
          int n = 0;
          auto accumulate = [&](const ConstEntry& e, float f, float iv) {
            n += acc_entry<ORDER, ICI>(a, e, f, iv) ? 1 : 0;
          };
          walk_stencil(K, lds, regs, u, v, c, par, m, accumulate);
          n_first = n;
        } else {
          auto accumulate = [&](const ConstEntry& e, float f, float iv) { acc_entry<ORDER, ICI>(a, e, f, iv); };
          walk_stencil(K, lds, regs, u, v, c, par, m, accumulate);
        }
      } else if (m == 0) {
        int n = 0;
        auto accumulate = [&](float dx, float dy, float f, float iv, int s) {
          n += acc_sample<ORDER, ICI, STEER, TEMP>(a, dx, dy, f, iv, eedge, reach2, sc, TEMP ? K.s[s].kt[m] : 1.f)
                   ? 1
                   : 0;
        };
        walk_support<STEER, RAW16>(K, lds, regs, Xj, Yj, c, cls, m, sb, accumulate);
        n_first = n;
      } else {
        auto accumulate = [&](float dx, float dy, float f, float iv, int s) {
          acc_sample<ORDER, ICI, STEER, TEMP>(a, dx, dy, f, iv, eedge, reach2, sc, TEMP ? K.s[s].kt[m] : 1.f);
        };
        walk_support<STEER, RAW16>(K, lds, regs, Xj, Yj, c, cls, m, sb, accumulate);
      }

      // Once every lane of the wave has a valid top-order fit at some radius,
      // the output is that order's ICI result: the lower orders (kept only
      // for fallback) are no longer solved.
      const bool lower = __builtin_amdgcn_ballot_w64(!st[ORDER].any) != 0;
      Fits<float, ORDER> fr;
      solve_fits<float, ORDER, ICI, true>(a.m, a.b, a.B, K.tau_inv, lower, fr, a.f2, a.siv, a.sivf,
                                          float2{K.sc[m].edge_coef[cls], K.sc[m].mono_r[cls] * stretch});
      // The top order's rounding risk, formed here: the empty asm keeps the
      // compiler from sinking the bound's arithmetic (and with it the factors
      // it reads) past the FP64 pass below.
      float risk_top = fr.s[ORDER] / fmaxf(fabsf(fr.y[ORDER]), K.value_floor);
      asm volatile("" : "+v"(risk_top));
      bool x64[ORDER + 1];
#pragma unroll
      for (int o = 0; o <= ORDER; ++o) x64[o] = false;
      if constexpr (ORDER >= 1) {
        // Validity where the FP32 pivot cannot certify it (rho < the bound
        // kPivotCertifiesN) needs the support size N and, if N >= n_o, the
        // pivots of the normal matrix accumulated in FP64.  A counted support
        // smaller than n_o decides the fit at once.  Fits decided on FP64
        // pivots, and valid fits with rho < tau_fp64, take their value and
        // variance from the FP64 moments too.
        constexpr int nb_tab[3] = {1, 3, 6};
        bool small[ORDER + 1], dbl[ORDER + 1];
        small[0] = dbl[0] = false;
        bool any_dbl = false;
#pragma unroll
        for (int o = 1; o <= ORDER; ++o) {
          const bool used = o == ORDER || lower;
          bool sm = used && fr.rho[o] < kPivotCertifiesN;
          if (sm && n_first >= 0 && n_first < nb_tab[o]) {
            fr.ok[o] = false;
            sm = false;
          }
          small[o] = sm;
          dbl[o] = sm || (K.use_fp64 && used && fr.ok[o] && fr.rho[o] < K.tau_fp64);
          any_dbl = any_dbl || dbl[o];
        }
        // A second pass over the samples, taken by the whole wave when any
        // lane needs it, accumulates the normal matrix in FP64 (the order-2
        // sums only where an order-2 fit needs them) and counts the support.
        // The fits it redoes then take C0 = sum_k (g . phi_k) w_k f_k and
        // var C0 = sum_k (g . phi_k)^2 K_k w_k (positive terms: the moment
        // form g^T B g cancels badly at small pivots) from a third pass, with
        // g from the FP64 solve.
        if (__builtin_amdgcn_ballot_w64(any_dbl) != 0) {
          const bool hi = ORDER >= 2 && __builtin_amdgcn_ballot_w64(dbl[ORDER]) != 0;
          Acc64<ORDER> a64;
          acc64_zero(a64);
          int n = 0;
          auto second = [&](float dx, float dy, float f, float iv, int s) {
            (void)f;
            const float r2 = window_r2<STEER>(dx, dy, dx * dx, dy * dy, sc);
            if (r2 < reach2) {
              float kw = __builtin_amdgcn_fmed3f(__builtin_amdgcn_exp2f(-r2) - eedge, 0.f, 1.f);
              if constexpr (TEMP) kw *= K.s[s].kt[m];
              const float w = kw * iv;
              n += (w > 0.f) ? 1 : 0;
              acc64_sample<ORDER, false>(a64, dx, dy, 0.f, w, hi);
            }
          };
          walk_support<STEER, RAW16>(K, lds, regs, Xj, Yj, c, cls, m, sb, second);
          Fit64<ORDER> r64;
          if (hi) solve64<ORDER, ORDER, false>(a64, dbl, r64);
          else solve64<ORDER, 1, false>(a64, dbl, r64);  // only order-1 fits to redo
          bool redo[ORDER + 1];
          bool any_redo = false;
          redo[0] = false;
#pragma unroll
          for (int o = 1; o <= ORDER; ++o) {
            if (small[o]) {
              fr.rho[o] = (float)r64.rho[o];
              fr.ok[o] = r64.rho[o] >= (double)K.tau_inv && n >= nb_tab[o];
            }
            redo[o] = dbl[o] && fr.ok[o];
            any_redo = any_redo || redo[o];
          }
          if (__builtin_amdgcn_ballot_w64(any_redo) != 0) {
            double ys[ORDER + 1];
            float vs[ORDER + 1];
#pragma unroll
            for (int o = 0; o <= ORDER; ++o) {
              ys[o] = 0.0;
              vs[o] = 0.f;
            }
            auto third = [&](float dx, float dy, float f, float iv, int s) {
              const float x2 = dx * dx, y2 = dy * dy;
              const float r2 = window_r2<STEER>(dx, dy, x2, y2, sc);
              if (r2 < reach2) {
                float kw = __builtin_amdgcn_fmed3f(__builtin_amdgcn_exp2f(-r2) - eedge, 0.f, 1.f);
                if constexpr (TEMP) kw *= K.s[s].kt[m];
                const float w = kw * iv;
                const double x = dx, y = dy, wf = (double)w * (double)f;
                const double phi[6] = {1.0, x, y, x * x, x * y, y * y};
#pragma unroll
                for (int o = 1; o <= ORDER; ++o) {
                  double t = r64.g[o][0];
#pragma unroll
                  for (int i = 1; i < nb_tab[o]; ++i) t = __builtin_fma(r64.g[o][i], phi[i], t);
                  ys[o] = __builtin_fma(t, wf, ys[o]);
                  if constexpr (ICI) {
                    const float tf = (float)t;
                    vs[o] = __builtin_fmaf(tf * tf, w * kw, vs[o]);
                  }
                }
              }
            };
            walk_support<STEER, RAW16>(K, lds, regs, Xj, Yj, c, cls, m, sb, third);
#pragma unroll
            for (int o = 1; o <= ORDER; ++o) {
              if (redo[o]) {
                fr.y[o] = (float)ys[o];
                if constexpr (ICI) fr.v[o] = vs[o];
                x64[o] = true;
              }
            }
          }
        }
      }
#pragma unroll
      for (int o = 0; o <= ORDER; ++o)
        if (o == ORDER || lower)
          ici_step(st[o], fr.ok[o], fr.y[o], fr.v[o], K.gamma, m,
                   (o == ORDER && !x64[o]) ? risk_top : __builtin_inff());
    }

    // the chosen order (highest with a valid fit) and its ICI result
    float val = __builtin_nanf(""), sdc = __builtin_nanf("");
    uint8_t cd = 0xFF;
    int mc = -1;
    float risk = 0.f;
#pragma unroll
    for (int o = ORDER; o >= 0; --o) {
      if (cd == 0xFF && st[o].any) {
        val = st[o].y;
        sdc = st[o].sd;
        cd = (uint8_t)((o << 4) | st[o].chosen);
        mc = st[o].chosen;
        risk = st[o].risk;
      }
    }
    // Outputs whose FP32 rounding bound exceeds the target are marked for the
    // FP64 refit launch (refit_kernel), which recomputes them at the chosen
    // radius and order from the raw frame.
    const bool refit = active && mc >= 0 && risk > K.risk_max;
    if (active) {
      if (K.refit_map) K.refit_map[(int64_t)v * K.refit_pitch + 3 * u + c] = refit ? (uint8_t)(0x80 | cd) : 0;
      cnt64 += refit ? 1 : 0;
      cnt_nan += cd == 0xFF ? 1 : 0;
    }
    // written as soon as the channel is done: nothing of it stays live
    // through the next channel's walks
    if (active) {
      float* orow = reinterpret_cast<float*>(reinterpret_cast<char*>(K.rgb) + (int64_t)v * K.rgb_pitch);
      orow[3 * u + c] = val;
      if (K.map) K.map[(int64_t)v * K.map_pitch + 3 * u + c] = cd;
      if (K.sd) {
        float* srow = reinterpret_cast<float*>(reinterpret_cast<char*>(K.sd) + (int64_t)v * K.sd_pitch);
        srow[3 * u + c] = sdc;
      }
    }
  }
}

// Per-workgroup LDS beside the staged samples.
struct TileShared {
  Region regs[kMaxSensors];
  uint32_t stat[2];  // the tile's FP64-valued and no-data outputs
};

template <int ORDER, bool ICI, int SRC, bool STEER = false, bool STENCIL = false, bool TEMP = false,
          bool RAW16 = false>
__device__ __forceinline__ void process_tile(const LaunchK& K, int tile, float2* lds, TileShared& sh) {
  const int tx = tile % K.tiles_x;
  const int ty = tile / K.tiles_x;
  const int u0 = tx * K.tile_w, v0 = ty * K.tile_h;
  const int tid = threadIdx.x;
  const int nthreads = K.tile_w * K.tile_h;
  if (tid < 2) sh.stat[tid] = 0u;
  if constexpr (RAW16) stage_tile_raw16(K, u0, v0, reinterpret_cast<uint16_t*>(lds), sh.regs, tid, nthreads);
  else stage_tile<SRC, STENCIL>(K, u0, v0, lds, sh.regs, tid, nthreads);
  __syncthreads();
  int du, dv;
  lane_pixel(tid, K.tile_w, K.tile_h, &du, &dv);
  const int u = u0 + du, v = v0 + dv;
  const bool active = (u < K.out_w) && (v < K.out_h);
  // inactive lanes of a ragged tile compute at their nominal pixel (staged)
  int cnt64 = 0, cnt_nan = 0;
  fit_pixel<ORDER, ICI, STEER, STENCIL, TEMP, RAW16>(K, lds, sh.regs, u, v, active, cnt64, cnt_nan);
  if (K.tile_stats) {
    if (cnt64) atomicAdd(&sh.stat[0], (uint32_t)cnt64);
    if (cnt_nan) atomicAdd(&sh.stat[1], (uint32_t)cnt_nan);
    __syncthreads();
    if (tid == 0) {
      K.tile_stats[2 * tile] = sh.stat[0];
      K.tile_stats[2 * tile + 1] = sh.stat[1];
    }
  }
}


// Compiled for at least 3 waves per SIMD (<= 168 VGPRs).
template <int ORDER, bool ICI, int SRC>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 8))) fit_kernel(const LaunchK K) {
  extern __shared__ float2 lds[];
  __shared__ TileShared sh;
  process_tile<ORDER, ICI, SRC>(K, xcd_tile(blockIdx.x, gridDim.x), lds, sh);
}

// Same kernel compiled for 4 waves per SIMD (<= 128 VGPRs: some values spill
// to scratch around each window walk, outside the per-sample loop); the tuner
// picks whichever is faster for a frame's class.
template <int ORDER, bool ICI, int SRC>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8)))
fit_kernel_occ4(const LaunchK K) {
  extern __shared__ float2 lds[];
  __shared__ TileShared sh;
  process_tile<ORDER, ICI, SRC>(K, xcd_tile(blockIdx.x, gridDim.x), lds, sh);
}

// Temporal LPA: the launch's sensors are the rig's sensors at several frames
// (one staged region each), every sample's window scaled by its frame's
// temporal factor.
template <int ORDER, bool ICI, int SRC>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 8)))
fit_kernel_temporal(const LaunchK K) {
  extern __shared__ float2 lds[];
  __shared__ TileShared sh;
  process_tile<ORDER, ICI, SRC, false, false, true>(K, xcd_tile(blockIdx.x, gridDim.x), lds, sh);
}

// The same with the tile staged as raw 16-bit DN (frames of 16-bit raw
// without calibration frames): a quarter of the LDS, and with it more
// workgroups per CU for the many staged sensors of a temporal support; then
// registers bound the occupancy, and 4 waves per SIMD (a few spilled) beat 3.
template <int ORDER, bool ICI>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8)))
fit_kernel_temporal_raw16(const LaunchK K) {
  extern __shared__ float2 lds[];
  __shared__ TileShared sh;
  process_tile<ORDER, ICI, SRC_RAW_U16, false, false, true, true>(K, xcd_tile(blockIdx.x, gridDim.x), lds, sh);
}

// ---------------------------------------------------------------------------
// Adaptive anisotropic LPA with colour-channel correlation (Sec. 5.4, 5.5).
// ---------------------------------------------------------------------------

// Fit with per-pixel steered windows (the boxes cover the stretched ellipse).
template <int ORDER, bool ICI, int SRC>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 8)))
fit_kernel_steer(const LaunchK K) {
  extern __shared__ float2 lds[];
  __shared__ TileShared sh;
  process_tile<ORDER, ICI, SRC, true>(K, xcd_tile(blockIdx.x, gridDim.x), lds, sh);
}

// Fit with pre-computed window weights (translation-only rigs, 256-lane
// tiles): the per-sample work is the moment FMAs alone.  Two register
// budgets, 3 and 4 waves per SIMD (the launch descriptor's occupancy picks).
template <int ORDER, bool ICI, int SRC>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 8)))
fit_kernel_stencil(const LaunchK K) {
  extern __shared__ float2 lds[];
  __shared__ TileShared sh;
  process_tile<ORDER, ICI, SRC, false, true>(K, xcd_tile(blockIdx.x, gridDim.x), lds, sh);
}

template <int ORDER, bool ICI, int SRC>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8)))
fit_kernel_stencil_occ4(const LaunchK K) {
  extern __shared__ float2 lds[];
  __shared__ TileShared sh;
  process_tile<ORDER, ICI, SRC, false, true>(K, xcd_tile(blockIdx.x, gridDim.x), lds, sh);
}

// Full coefficient vector of one fit in FP64: LDL^T of A (as in solve_fits),
// then A C = b.  Returns C1 = (C[1], C[2]), the smallest equilibrated pivot
// and whether every diagonal entry is positive.
template <int ORDER>
__device__ __forceinline__ void solve_gradient(const double* m, const double* b, double& c1x, double& c1y,
                                               double& rho, bool& diag_all) {
  constexpr int NB = n_basis<ORDER>();
  double L[NB][NB], U[NB][NB], iD[NB];
  rho = 1e300;
  diag_all = true;
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    const double ajj = m[aidx(j, j)];
    diag_all = diag_all && ajj > 0.0;
    double d = ajj;
#pragma unroll
    for (int k = 0; k < j; ++k) d -= U[j][k] * L[j][k];
    iD[j] = d > 0.0 ? 1.0 / d : 0.0;
    const double req = ajj > 0.0 ? d / ajj : 0.0;
    rho = req < rho ? req : rho;
#pragma unroll
    for (int i = j + 1; i < NB; ++i) {
      double t = m[aidx(i, j)];
#pragma unroll
      for (int k = 0; k < j; ++k) t -= U[i][k] * L[j][k];
      U[i][j] = t;
      L[i][j] = t * iD[j];
    }
  }
  double z[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    double t = b[i];
#pragma unroll
    for (int k = 0; k < i; ++k) t -= L[i][k] * z[k];
    z[i] = t;
  }
  double C[NB];
#pragma unroll
  for (int i = NB - 1; i >= 0; --i) {
    double t = z[i] * iD[i];
#pragma unroll
    for (int k = i + 1; k < NB; ++k) t -= L[k][i] * C[k];
    C[i] = t;
  }
  c1x = C[1];
  c1y = C[2];
  if (!diag_all || !(rho > 0.0)) rho = 0.0;
}

// Gradient pass (Sec. 5.4 first step, G channel as in Sec. 5.5): isotropic
// order-1 or order-2 fit of the G channel at radius K.sc[0]; its C1 in
// reference-plane units (the fit ran in coordinates scaled by s), zero where
// the fit is invalid.  Its moments are accumulated and solved in FP64: every
// gradient feeds the steering of the (2q+1)^2 pixels around it, and FP32
// rounding of an ill-conditioned gradient fit would move all their windows.
// The pass is one channel at one radius, a small part of the whole.
template <int ORDER, int SRC>
__global__ void __launch_bounds__(256) grad_kernel(const LaunchK K) {
  extern __shared__ float2 lds[];
  __shared__ Region regs[kMaxSensors];
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int u0 = (tile % K.tiles_x) * K.tile_w, v0 = (tile / K.tiles_x) * K.tile_h;
  const int tid = threadIdx.x;
  stage_tile<SRC>(K, u0, v0, lds, regs, tid, K.tile_w * K.tile_h);
  __syncthreads();
  int du, dv;
  lane_pixel(tid, K.tile_w, K.tile_h, &du, &dv);
  const int u = u0 + du, v = v0 + dv;
  const bool active = (u < K.out_w) && (v < K.out_h);
  const double Xj = K.out_affine[0] * u + K.out_affine[1] * v + K.out_affine[2];
  const double Yj = K.out_affine[3] * u + K.out_affine[4] * v + K.out_affine[5];
  const float eedge = K.sc[0].e_edge[1];
  const float reach2 = K.sc[0].reach2[1];
  double m64[n_mom<ORDER>()], b64[n_basis<ORDER>()];
#pragma unroll
  for (int k = 0; k < n_mom<ORDER>(); ++k) m64[k] = 0.0;
#pragma unroll
  for (int k = 0; k < n_basis<ORDER>(); ++k) b64[k] = 0.0;
  int n = 0;
  auto accumulate = [&](float dx, float dy, float f, float iv, int s) {
    const float r2 = dx * dx + dy * dy;
    if (r2 < reach2) {
      const float w = fmaxf(__builtin_amdgcn_exp2f(-r2) - eedge, 0.f) * iv;
      n += (w > 0.f) ? 1 : 0;
      const double wd = w, x = dx, y = dy, wf = wd * (double)f;
      const double xx = x * x, xy = x * y, yy = y * y;
      m64[0] += wd;
      m64[1] += wd * x;
      m64[2] += wd * y;
      m64[3] += wd * xx;
      m64[4] += wd * xy;
      m64[5] += wd * yy;
      b64[0] += wf;
      b64[1] += wf * x;
      b64[2] += wf * y;
      if constexpr (ORDER >= 2) {
        m64[6] += wd * xx * x;
        m64[7] += wd * xx * y;
        m64[8] += wd * xy * y;
        m64[9] += wd * yy * y;
        m64[10] += wd * xx * xx;
        m64[11] += wd * xx * xy;
        m64[12] += wd * xx * yy;
        m64[13] += wd * xy * yy;
        m64[14] += wd * yy * yy;
        b64[3] += wf * xx;
        b64[4] += wf * xy;
        b64[5] += wf * yy;
      }
    }
  };
  walk_support<false>(K, lds, regs, Xj, Yj, 1, 1, 0, SteerBox{}, accumulate);
  double c1x, c1y, rho;
  bool diag_all;
  solve_gradient<ORDER>(m64, b64, c1x, c1y, rho, diag_all);
  const bool ok = diag_all && rho >= (double)K.tau_inv && n >= n_basis<ORDER>();
  if (active) {
    const double s = K.sc[0].coord_scale[1];
    float2* row = reinterpret_cast<float2*>(reinterpret_cast<char*>(K.grad) + (int64_t)v * K.grad_pitch);
    row[u] = ok ? make_float2((float)(c1x * s), (float)(c1y * s)) : make_float2(0.f, 0.f);
  }
}

// Steering pass (Sec. 5.4): the gradients of the (2q+1)^2 output pixels around
// (u, v) inside the grid form G; the eigen-decomposition of G^T G gives its
// singular values s1 >= s2 and the dominant gradient direction u1.  The
// steering matrix C = gamma U diag(sigma, 1/sigma) U^T has eigenvalue
// gamma*sigma along u1 (across the edge) and gamma/sigma along the edge, each
// clamped to [lo, hi]; it is formed as lb I + (la - lb) u1 u1^T.  FP64: the
// near-rank-1 structure tensors of edges would lose s2 to cancellation.
__global__ void __launch_bounds__(256) steer_kernel(const SteerArgs A) {
  const int u = blockIdx.x * 16 + (threadIdx.x & 15);
  const int v = blockIdx.y * 16 + (threadIdx.x >> 4);
  if (u >= A.out_w || v >= A.out_h) return;
  double txx = 0.0, txy = 0.0, tyy = 0.0;
  int count = 0;
  for (int b = -A.q; b <= A.q; ++b) {
    const int vv = v + b;
    if (vv < 0 || vv >= A.out_h) continue;
    const float2* row = reinterpret_cast<const float2*>(reinterpret_cast<const char*>(A.grad) + (int64_t)vv * A.grad_pitch);
    for (int a = -A.q; a <= A.q; ++a) {
      const int uu = u + a;
      if (uu < 0 || uu >= A.out_w) continue;
      const float2 g = row[uu];
      const double gx = g.x, gy = g.y;
      txx += gx * gx;
      txy += gx * gy;
      tyy += gy * gy;
      ++count;
    }
  }
  const double half_tr = 0.5 * (txx + tyy);
  const double disc = sqrt(0.25 * (txx - tyy) * (txx - tyy) + txy * txy);
  const double e1 = half_tr + disc;
  const double e2 = half_tr - disc > 0.0 ? half_tr - disc : 0.0;
  const double s1 = sqrt(e1), s2 = sqrt(e2);
  const double phi = 0.5 * atan2(2.0 * txy, txx - tyy);
  const double ux = cos(phi), uy = sin(phi);
  const double sigma = (s1 + A.lambda1) / (s2 + A.lambda1);
  const double gamma = pow((s1 * s2 + A.lambda2) / (double)count, A.alpha);
  double la = gamma * sigma, lb = gamma / sigma;
  la = la < A.lo ? A.lo : (la > A.hi ? A.hi : la);
  lb = lb < A.lo ? A.lo : (lb > A.hi ? A.hi : lb);
  float4* out = reinterpret_cast<float4*>(reinterpret_cast<char*>(A.steer) + (int64_t)v * A.steer_pitch);
  out[u] = make_float4((float)(lb + (la - lb) * ux * ux), (float)((la - lb) * ux * uy),
                       (float)(lb + (la - lb) * uy * uy), 0.f);
}

// Persistent form: the batch's tiles (frame-major, each frame's tiles
// row-major) are split into kXcds contiguous ranges with a device counter
// each.  A workgroup first takes tiles from the range of its own XCD
// (workgroups are dispatched to the XCDs round-robin), so neighbouring tiles
// share that XCD's L2, then from the other ranges in turn until all are
// exhausted.  It moves to the next range only when a claim fails, at most
// kXcds times, so every workgroup reaches the exit.  The frame's order and
// single/multi-radius class select the fit code per tile (a
// workgroup-uniform branch); all frames of one launch share SRC.  Compiled for
// 4 waves per SIMD: order-2 tiles spill a few values around their solves, as
// in fit_kernel_occ4, and the batch still runs faster than at 3 waves.
template <int SRC>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8))) fit_batch_kernel(const BatchHeader* __restrict__ hdr,
                                                       const LaunchK* __restrict__ frames,
                                                       const int64_t* __restrict__ first_tile,
                                                       int* __restrict__ queue) {
  extern __shared__ float2 lds[];
  __shared__ TileShared sh;
  __shared__ int next_tile;
  const int n_frames = hdr->n_frames;
  const int64_t total_tiles = hdr->total_tiles;
  int range = blockIdx.x % kXcds, failed = 0;  // used by thread 0 only
  for (;;) {
    if (threadIdx.x == 0) {
      int t = -1;
      while (failed < kXcds) {
        const int64_t lo = total_tiles * range / kXcds, hi = total_tiles * (range + 1) / kXcds;
        const int64_t c = lo + atomicAdd(&queue[range], 1);
        if (c < hi) {
          t = (int)c;
          break;
        }
        range = (range + 1) % kXcds;
        ++failed;
      }
      next_tile = t;
    }
    __syncthreads();
    const int t = next_tile;
    __syncthreads();
    if (t < 0) break;
    // frame owning global tile t (binary search over first-tile offsets)
    int lo = 0, hi = n_frames - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (first_tile[mid] <= t) lo = mid; else hi = mid - 1;
    }
    const int f = __builtin_amdgcn_readfirstlane(lo);
    const LaunchK& K = frames[f];
    const int local = (int)(t - first_tile[f]);
    switch (K.order * 2 + (K.need_var ? 1 : 0)) {
      case 0: process_tile<0, false, SRC>(K, local, lds, sh); break;
      case 1: process_tile<0, true, SRC>(K, local, lds, sh); break;
      case 2: process_tile<1, false, SRC>(K, local, lds, sh); break;
      case 3: process_tile<1, true, SRC>(K, local, lds, sh); break;
      case 4: process_tile<2, false, SRC>(K, local, lds, sh); break;
      default: process_tile<2, true, SRC>(K, local, lds, sh); break;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Pre-pass: raw -> (radiance, inverse variance) FP32 plane, or raw -> FP16
// normalised value (y - 2^(bits-1)) 2^-bits, round-to-nearest-even (exact for
// raw values of up to 12 bits), +Inf masked.
// ---------------------------------------------------------------------------
template <bool RAW_F32, bool TO_F16>
__global__ void __launch_bounds__(256) prepass_kernel(const SensorK S, const void* raw, int64_t raw_pitch,
                                                      void* plane, int64_t plane_pitch, float norm_encode) {
  const int x = blockIdx.x * 64 + (threadIdx.x & 63);
  const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (x >= S.width || y >= S.height) return;
  const char* rrow = static_cast<const char*>(raw) + (int64_t)y * raw_pitch;
  const float dn = RAW_F32 ? reinterpret_cast<const float*>(rrow)[x]
                           : (float)reinterpret_cast<const uint16_t*>(rrow)[x];
  char* prow = static_cast<char*>(plane) + (int64_t)y * plane_pitch;
  const bool cal = S.calib != nullptr;
  const float4 c = cal ? S.calib[(int64_t)y * S.width + x] : make_float4(S.black, S.inv_ge, S.read_var, S.sat);
  if constexpr (TO_F16) {
    const __half h = (dn < c.w) ? __float2half_rn((dn - S.norm_offset) * norm_encode)
                                : __ushort_as_half((unsigned short)0x7C00u);
    reinterpret_cast<__half*>(prow)[x] = h;
  } else {
    reinterpret_cast<float2*>(prow)[x] = cal ? decode_dn_cal(S, dn, c) : decode_dn(S, dn);
  }
}

// The pre-pass of a whole batch (plane storage forms), one launch inside the
// batch graph: workgroup row blockIdx.y is frame y / kMaxSensors, sensor
// y % kMaxSensors of the batch table; its workgroups take bands of
// kPreRows rows (band blockIdx.x, then every gridDim.x-th).  Reads each
// frame's raw plane (S.raw) and writes the plane the fit reads (S.src,
// allocated by the library for this launch).  Where both planes' rows are
// 16-byte aligned, a lane converts 8 consecutive samples of every row of the
// band, with all the band's loads issued before the first conversion (16-byte
// loads and stores; the work is latency-bound with one sample per load).
constexpr int kPreRows = 4;

template <bool TO_F16>
__device__ __forceinline__ void prepass_one(const SensorK& S, float dn, float4 c, char* prow, int x) {
  if constexpr (TO_F16) {
    const float norm_encode = 1.f / S.norm_decode;  // a power of two: exact
    reinterpret_cast<__half*>(prow)[x] = (dn < c.w) ? __float2half_rn((dn - S.norm_offset) * norm_encode)
                                                    : __ushort_as_half((unsigned short)0x7C00u);
  } else {
    reinterpret_cast<float2*>(prow)[x] = (S.calib != nullptr) ? decode_dn_cal(S, dn, c) : decode_dn(S, dn);
  }
}

template <bool TO_F16>
__global__ void __launch_bounds__(256) prepass_batch_kernel(const BatchHeader* __restrict__ hdr,
                                                            const LaunchK* __restrict__ frames) {
  const int f = blockIdx.y / kMaxSensors, s = blockIdx.y % kMaxSensors;
  if (f >= hdr->n_frames) return;
  const LaunchK& K = frames[f];
  if (s >= K.n_sensors) return;
  const SensorK& S = K.s[s];
  const bool raw_f32 = S.raw_f32 != 0;
  const bool cal = S.calib != nullptr;
  const float4 c0 = make_float4(S.black, S.inv_ge, S.read_var, S.sat);
  const bool vec = ((reinterpret_cast<uintptr_t>(S.raw) | (uintptr_t)S.raw_pitch |
                     reinterpret_cast<uintptr_t>(S.src) | (uintptr_t)S.pitch) & 15) == 0;
  const int W = S.width, H = S.height;
  const int w8 = vec ? (W & ~7) : 0;  // samples converted 8 at a time
  for (int y0 = kPreRows * blockIdx.x; y0 < H; y0 += kPreRows * gridDim.x) {
    const int nr = min(kPreRows, H - y0);
    for (int x0 = 8 * threadIdx.x; x0 < w8; x0 += 8 * 256) {
      float dn[kPreRows][8];
#pragma unroll
      for (int r = 0; r < kPreRows; ++r) {
        if (r < nr) {
          const char* rrow = static_cast<const char*>(S.raw) + (int64_t)(y0 + r) * S.raw_pitch;
          if (raw_f32) {
            const float4 a = reinterpret_cast<const float4*>(rrow)[x0 >> 2];
            const float4 b = reinterpret_cast<const float4*>(rrow)[(x0 >> 2) + 1];
            dn[r][0] = a.x; dn[r][1] = a.y; dn[r][2] = a.z; dn[r][3] = a.w;
            dn[r][4] = b.x; dn[r][5] = b.y; dn[r][6] = b.z; dn[r][7] = b.w;
          } else {
            const uint4 q = reinterpret_cast<const uint4*>(rrow)[x0 >> 3];
            const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              dn[r][2 * k] = (float)(w[k] & 0xFFFFu);
              dn[r][2 * k + 1] = (float)(w[k] >> 16);
            }
          }
        }
      }
#pragma unroll
      for (int r = 0; r < kPreRows; ++r) {
        if (r < nr) {
          const int y = y0 + r;
          char* prow = static_cast<char*>(const_cast<void*>(S.src)) + (int64_t)y * S.pitch;
          float4 c[8];
#pragma unroll
          for (int k = 0; k < 8; ++k) c[k] = cal ? S.calib[(int64_t)y * W + x0 + k] : c0;
          if constexpr (TO_F16) {
            const float norm_encode = 1.f / S.norm_decode;  // a power of two: exact
            uint32_t w[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              const float d0 = dn[r][2 * k], d1 = dn[r][2 * k + 1];
              const __half h0 = (d0 < c[2 * k].w) ? __float2half_rn((d0 - S.norm_offset) * norm_encode)
                                                  : __ushort_as_half((unsigned short)0x7C00u);
              const __half h1 = (d1 < c[2 * k + 1].w) ? __float2half_rn((d1 - S.norm_offset) * norm_encode)
                                                      : __ushort_as_half((unsigned short)0x7C00u);
              w[k] = (uint32_t)__half_as_ushort(h0) | ((uint32_t)__half_as_ushort(h1) << 16);
            }
            reinterpret_cast<uint4*>(prow)[x0 >> 3] = make_uint4(w[0], w[1], w[2], w[3]);
          } else {
            float2 v[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) v[k] = cal ? decode_dn_cal(S, dn[r][k], c[k]) : decode_dn(S, dn[r][k]);
            float4* o = reinterpret_cast<float4*>(prow) + (x0 >> 1);
#pragma unroll
            for (int k = 0; k < 4; ++k) o[k] = make_float4(v[2 * k].x, v[2 * k].y, v[2 * k + 1].x, v[2 * k + 1].y);
          }
        }
      }
    }
    // the samples past the last group of 8 (all of them where rows are not aligned)
    for (int r = 0; r < nr; ++r) {
      const int y = y0 + r;
      const char* rrow = static_cast<const char*>(S.raw) + (int64_t)y * S.raw_pitch;
      char* prow = static_cast<char*>(const_cast<void*>(S.src)) + (int64_t)y * S.pitch;
      for (int x = w8 + threadIdx.x; x < W; x += 256) {
        const float dn = raw_f32 ? reinterpret_cast<const float*>(rrow)[x]
                                 : (float)reinterpret_cast<const uint16_t*>(rrow)[x];
        prepass_one<TO_F16>(S, dn, cal ? S.calib[(int64_t)y * W + x] : c0, prow, x);
      }
    }
  }
}

}  // namespace lpa

using namespace lpa;

namespace {
constexpr int kMaxLdsBytes = 64 * 1024;

template <int ORDER, bool ICI, int SRC>
void launch_fit_one(const LaunchK& K, dim3 grid, dim3 block, size_t lds, hipStream_t st) {
  if constexpr (ORDER == 2) {
    if (K.occupancy == 4) {
      fit_kernel_occ4<ORDER, ICI, SRC><<<grid, block, lds, st>>>(K);
      return;
    }
  }
  fit_kernel<ORDER, ICI, SRC><<<grid, block, lds, st>>>(K);
}

template <int ORDER, bool ICI>
int launch_fit_src(const LaunchK& K, hipStream_t st) {
  const dim3 grid(K.tiles_x * K.tiles_y), block(K.tile_w * K.tile_h);
  const size_t lds = (size_t)K.lds_floats2 * sizeof(float2);
  switch (K.src_kind) {
    case SRC_RAW_U16: launch_fit_one<ORDER, ICI, SRC_RAW_U16>(K, grid, block, lds, st); break;
    case SRC_RAW_F32: launch_fit_one<ORDER, ICI, SRC_RAW_F32>(K, grid, block, lds, st); break;
    case SRC_PLANE_F32: launch_fit_one<ORDER, ICI, SRC_PLANE_F32>(K, grid, block, lds, st); break;
    case SRC_PLANE_F16: launch_fit_one<ORDER, ICI, SRC_PLANE_F16>(K, grid, block, lds, st); break;
    default: return -1;
  }
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

// Every sensor of a fit launch must name its raw plane (the FP64 refit reads it).
bool raw_bound(const LaunchK& K) {
  for (int s = 0; s < K.n_sensors; ++s)
    if (!K.s[s].raw) return false;
  return true;
}

}  // namespace

extern "C" int lpa_k_fit_max_lds_bytes(void) { return kMaxLdsBytes; }

extern "C" int lpa_k_grad(const LaunchK* k, void* stream) {
  const LaunchK& K = *k;
  if (K.tile_w * K.tile_h > 256 || (size_t)K.lds_floats2 * sizeof(float2) > (size_t)kMaxLdsBytes) return -1;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const dim3 grid(K.tiles_x * K.tiles_y), block(K.tile_w * K.tile_h);
  const size_t lds = (size_t)K.lds_floats2 * sizeof(float2);
#define LPA_GRAD(O, S) grad_kernel<O, S><<<grid, block, lds, st>>>(K)
  if (K.order == 1) {
    switch (K.src_kind) {
      case SRC_RAW_U16: LPA_GRAD(1, SRC_RAW_U16); break;
      case SRC_RAW_F32: LPA_GRAD(1, SRC_RAW_F32); break;
      case SRC_PLANE_F32: LPA_GRAD(1, SRC_PLANE_F32); break;
      case SRC_PLANE_F16: LPA_GRAD(1, SRC_PLANE_F16); break;
      default: return -1;
    }
  } else if (K.order == 2) {
    switch (K.src_kind) {
      case SRC_RAW_U16: LPA_GRAD(2, SRC_RAW_U16); break;
      case SRC_RAW_F32: LPA_GRAD(2, SRC_RAW_F32); break;
      case SRC_PLANE_F32: LPA_GRAD(2, SRC_PLANE_F32); break;
      case SRC_PLANE_F16: LPA_GRAD(2, SRC_PLANE_F16); break;
      default: return -1;
    }
  } else {
    return -1;
  }
#undef LPA_GRAD
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

extern "C" int lpa_k_steer(const SteerArgs* a, void* stream) {
  const dim3 grid((a->out_w + 15) / 16, (a->out_h + 15) / 16), block(256);
  steer_kernel<<<grid, block, 0, static_cast<hipStream_t>(stream)>>>(*a);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

namespace {
template <int ORDER, bool ICI>
int launch_steer_src(const LaunchK& K, hipStream_t st) {
  const dim3 grid(K.tiles_x * K.tiles_y), block(K.tile_w * K.tile_h);
  const size_t lds = (size_t)K.lds_floats2 * sizeof(float2);
  switch (K.src_kind) {
    case SRC_RAW_U16: fit_kernel_steer<ORDER, ICI, SRC_RAW_U16><<<grid, block, lds, st>>>(K); break;
    case SRC_RAW_F32: fit_kernel_steer<ORDER, ICI, SRC_RAW_F32><<<grid, block, lds, st>>>(K); break;
    case SRC_PLANE_F32: fit_kernel_steer<ORDER, ICI, SRC_PLANE_F32><<<grid, block, lds, st>>>(K); break;
    case SRC_PLANE_F16: fit_kernel_steer<ORDER, ICI, SRC_PLANE_F16><<<grid, block, lds, st>>>(K); break;
    default: return -1;
  }
  return hipGetLastError() == hipSuccess ? 0 : -2;
}
}  // namespace

extern "C" int lpa_k_fit_steered(const LaunchK* k, void* stream) {
  const LaunchK& K = *k;
  if (!raw_bound(K) || !K.steer || K.tile_w * K.tile_h > 256 || (size_t)K.lds_floats2 * sizeof(float2) > (size_t)kMaxLdsBytes)
    return -1;
  hipStream_t st = static_cast<hipStream_t>(stream);
  switch (K.order * 2 + (K.need_var ? 1 : 0)) {
    case 0: return launch_steer_src<0, false>(K, st);
    case 1: return launch_steer_src<0, true>(K, st);
    case 2: return launch_steer_src<1, false>(K, st);
    case 3: return launch_steer_src<1, true>(K, st);
    case 4: return launch_steer_src<2, false>(K, st);
    case 5: return launch_steer_src<2, true>(K, st);
    default: return -1;
  }
}

namespace {
template <int ORDER, bool ICI, int SRC>
void launch_stencil_one(const LaunchK& K, dim3 grid, dim3 block, size_t lds, hipStream_t st) {
  if (K.occupancy == 4) fit_kernel_stencil_occ4<ORDER, ICI, SRC><<<grid, block, lds, st>>>(K);
  else fit_kernel_stencil<ORDER, ICI, SRC><<<grid, block, lds, st>>>(K);
}

template <int ORDER, bool ICI>
int launch_stencil_src(const LaunchK& K, hipStream_t st) {
  const dim3 grid(K.tiles_x * K.tiles_y), block(K.tile_w * K.tile_h);
  const size_t lds = (size_t)K.lds_floats2 * sizeof(float2);
  switch (K.src_kind) {
    case SRC_RAW_U16: launch_stencil_one<ORDER, ICI, SRC_RAW_U16>(K, grid, block, lds, st); break;
    case SRC_RAW_F32: launch_stencil_one<ORDER, ICI, SRC_RAW_F32>(K, grid, block, lds, st); break;
    case SRC_PLANE_F32: launch_stencil_one<ORDER, ICI, SRC_PLANE_F32>(K, grid, block, lds, st); break;
    case SRC_PLANE_F16: launch_stencil_one<ORDER, ICI, SRC_PLANE_F16>(K, grid, block, lds, st); break;
    default: return -1;
  }
  return hipGetLastError() == hipSuccess ? 0 : -2;
}
}  // namespace

extern "C" int lpa_k_fit_stencil(const LaunchK* k, void* stream) {
  const LaunchK& K = *k;
  // one parity class per wave needs 256-lane tiles
  if (!raw_bound(K) || !K.stencil || K.tile_w * K.tile_h != 256 || (size_t)K.lds_floats2 * sizeof(float2) > (size_t)kMaxLdsBytes)
    return -1;
  hipStream_t st = static_cast<hipStream_t>(stream);
  switch (K.order * 2 + (K.need_var ? 1 : 0)) {
    case 0: return launch_stencil_src<0, false>(K, st);
    case 1: return launch_stencil_src<0, true>(K, st);
    case 2: return launch_stencil_src<1, false>(K, st);
    case 3: return launch_stencil_src<1, true>(K, st);
    case 4: return launch_stencil_src<2, false>(K, st);
    case 5: return launch_stencil_src<2, true>(K, st);
    default: return -1;
  }
}

extern "C" int lpa_k_fit(const LaunchK* k, void* stream) {
  const LaunchK& K = *k;
  if (!raw_bound(K) || K.tile_w * K.tile_h > 256 || (size_t)K.lds_floats2 * sizeof(float2) > (size_t)kMaxLdsBytes) return -1;
  hipStream_t st = static_cast<hipStream_t>(stream);
  switch (K.order * 2 + (K.need_var ? 1 : 0)) {
    case 0: return launch_fit_src<0, false>(K, st);
    case 1: return launch_fit_src<0, true>(K, st);
    case 2: return launch_fit_src<1, false>(K, st);
    case 3: return launch_fit_src<1, true>(K, st);
    case 4: return launch_fit_src<2, false>(K, st);
    case 5: return launch_fit_src<2, true>(K, st);
    default: return -1;
  }
}

namespace {
template <int ORDER, bool ICI>
int launch_temporal_src(const LaunchK& K, hipStream_t st) {
  const dim3 grid(K.tiles_x * K.tiles_y), block(K.tile_w * K.tile_h);
  const size_t lds = (size_t)K.lds_floats2 * sizeof(float2);
  // the raw staging needs every sensor to mask 0xFFFF (no calibration
  // frames, saturation at most 65535 DN)
  bool raw16 = K.src_kind == SRC_RAW_U16;
  for (int s = 0; s < K.n_sensors; ++s) raw16 = raw16 && K.s[s].calib == nullptr && K.s[s].sat <= 65535.f;
  if (raw16) {
    const size_t lds16 = ((size_t)K.lds_floats2 * sizeof(uint16_t) + 15) / 16 * 16;
    fit_kernel_temporal_raw16<ORDER, ICI><<<grid, block, lds16, st>>>(K);
    return hipGetLastError() == hipSuccess ? 0 : -2;
  }
  switch (K.src_kind) {
    case SRC_RAW_U16: fit_kernel_temporal<ORDER, ICI, SRC_RAW_U16><<<grid, block, lds, st>>>(K); break;
    case SRC_RAW_F32: fit_kernel_temporal<ORDER, ICI, SRC_RAW_F32><<<grid, block, lds, st>>>(K); break;
    default: return -1;
  }
  return hipGetLastError() == hipSuccess ? 0 : -2;
}
}  // namespace

extern "C" int lpa_k_fit_temporal(const LaunchK* k, void* stream) {
  const LaunchK& K = *k;
  if (!raw_bound(K) || K.tile_w * K.tile_h > 256 || (size_t)K.lds_floats2 * sizeof(float2) > (size_t)kMaxLdsBytes) return -1;
  hipStream_t st = static_cast<hipStream_t>(stream);
  switch (K.order * 2 + (K.need_var ? 1 : 0)) {
    case 0: return launch_temporal_src<0, false>(K, st);
    case 1: return launch_temporal_src<0, true>(K, st);
    case 2: return launch_temporal_src<1, false>(K, st);
    case 3: return launch_temporal_src<1, true>(K, st);
    case 4: return launch_temporal_src<2, false>(K, st);
    case 5: return launch_temporal_src<2, true>(K, st);
    default: return -1;
  }
}

extern "C" int lpa_k_prepass(const SensorK* s, int raw_is_f32, const void* raw, int64_t raw_pitch,
                             void* plane, int64_t plane_pitch, int to_f16, float norm_encode,
                             void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  const dim3 grid((s->width + 63) / 64, (s->height + 3) / 4), block(256);
  if (raw_is_f32) {
    if (to_f16) prepass_kernel<true, true><<<grid, block, 0, st>>>(*s, raw, raw_pitch, plane, plane_pitch, norm_encode);
    else prepass_kernel<true, false><<<grid, block, 0, st>>>(*s, raw, raw_pitch, plane, plane_pitch, norm_encode);
  } else {
    if (to_f16) prepass_kernel<false, true><<<grid, block, 0, st>>>(*s, raw, raw_pitch, plane, plane_pitch, norm_encode);
    else prepass_kernel<false, false><<<grid, block, 0, st>>>(*s, raw, raw_pitch, plane, plane_pitch, norm_encode);
  }
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

extern "C" int lpa_k_fit_batch(const BatchHeader* d_hdr, const LaunchK* d_frames,
                               const int64_t* d_first_tile, int32_t* d_queue, int32_t src_kind,
                               int32_t block, int32_t lds_floats2, int32_t grid, void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  const size_t lds = (size_t)lds_floats2 * sizeof(float2);
  if (block > 256 || lds > (size_t)kMaxLdsBytes) return -1;
  switch (src_kind) {
    case SRC_RAW_U16: fit_batch_kernel<SRC_RAW_U16><<<grid, block, lds, st>>>(d_hdr, d_frames, d_first_tile, d_queue); break;
    case SRC_RAW_F32: fit_batch_kernel<SRC_RAW_F32><<<grid, block, lds, st>>>(d_hdr, d_frames, d_first_tile, d_queue); break;
    case SRC_PLANE_F32: fit_batch_kernel<SRC_PLANE_F32><<<grid, block, lds, st>>>(d_hdr, d_frames, d_first_tile, d_queue); break;
    case SRC_PLANE_F16: fit_batch_kernel<SRC_PLANE_F16><<<grid, block, lds, st>>>(d_hdr, d_frames, d_first_tile, d_queue); break;
    default: return -1;
  }
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

extern "C" int lpa_k_refit(const LaunchK* k, void* stream) {
  const LaunchK& K = *k;
  const bool f32 = K.s[0].raw_f32 != 0;
  const size_t lds = (size_t)K.refit_lds * (f32 ? 4 : 2);
  if (!K.refit_map || !raw_bound(K) || K.refit_bw < 1 || K.refit_bh < 1 || K.refit_bw * K.refit_bh * 3 > kRefitMaxOut ||
      lds > (size_t)lpa_k_refit_max_lds_bytes())
    return -1;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const dim3 grid(((K.out_w + K.refit_bw - 1) / K.refit_bw) * ((K.out_h + K.refit_bh - 1) / K.refit_bh)),
      block(kRefitThreads);
  const bool steer = K.steer != nullptr;
#define LPA_REFIT(O, ST)                                                          \
  (f32 ? (refit_kernel<O, ST, float><<<grid, block, lds, st>>>(K), 0)          \
       : (refit_kernel<O, ST, uint16_t><<<grid, block, lds, st>>>(K), 0))
  switch (K.order * 2 + (steer ? 1 : 0)) {
    case 0: LPA_REFIT(0, false); break;
    case 1: LPA_REFIT(0, true); break;
    case 2: LPA_REFIT(1, false); break;
    case 3: LPA_REFIT(1, true); break;
    case 4: LPA_REFIT(2, false); break;
    case 5: LPA_REFIT(2, true); break;
    default: return -1;
  }
#undef LPA_REFIT
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

extern "C" int lpa_k_refit_batch(const BatchHeader* hdr, const LaunchK* frames, const int64_t* first_tile,
                                 int32_t grid, int32_t lds_bytes, int32_t raw_f32, void* stream) {
  if (lds_bytes > lpa_k_refit_max_lds_bytes()) return -1;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (raw_f32) refit_batch_kernel<float><<<grid, kRefitThreads, (size_t)lds_bytes, st>>>(hdr, frames, first_tile);
  else refit_batch_kernel<uint16_t><<<grid, kRefitThreads, (size_t)lds_bytes, st>>>(hdr, frames, first_tile);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

// Dynamic LDS a refit launch may take: 64 KiB less its static arrays.
extern "C" int lpa_k_refit_max_lds_bytes(void) {
  return 64 * 1024 - (int)(sizeof(uint16_t) * kRefitMaxOut + sizeof(int) * (kRefitClasses + 1) +
                           sizeof(Region) * kMaxSensors + sizeof(int) * kMaxSensors) - 256;
}

namespace {
__global__ void zero_i32_kernel(int* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}
}  // namespace



namespace {
// One workgroup of 256 threads sums n pairs of per-tile counts.
__device__ void sum_pairs(const uint32_t* t, int64_t n, uint64_t* out) {
  __shared__ uint64_t part[2][256];
  uint64_t a = 0, b = 0;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    a += t[2 * i];
    b += t[2 * i + 1];
  }
  part[0][threadIdx.x] = a;
  part[1][threadIdx.x] = b;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      part[0][threadIdx.x] += part[0][threadIdx.x + w];
      part[1][threadIdx.x] += part[1][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = part[0][0];
    out[1] = part[1][0];
  }
}

__global__ void __launch_bounds__(256) stats_sum_kernel(const uint32_t* t, int64_t n, uint64_t* out) {
  sum_pairs(t, n, out);
}

__global__ void __launch_bounds__(256) stats_frames_kernel(const BatchHeader* hdr, const LaunchK* frames) {
  const int f = blockIdx.x;
  if (f >= hdr->n_frames) return;
  const LaunchK& K = frames[f];
  if (!K.tile_stats || !K.frame_stats) return;
  sum_pairs(K.tile_stats, (int64_t)K.tiles_x * K.tiles_y, K.frame_stats);
}
}  // namespace

extern "C" int lpa_k_stats_sum(const uint32_t* tile_stats, int64_t n_tiles, uint64_t* out, void* stream) {
  stats_sum_kernel<<<1, 256, 0, static_cast<hipStream_t>(stream)>>>(tile_stats, n_tiles, out);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

extern "C" int lpa_k_stats_frames(const BatchHeader* hdr, const LaunchK* frames, int32_t grid, void* stream) {
  stats_frames_kernel<<<grid, 256, 0, static_cast<hipStream_t>(stream)>>>(hdr, frames);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

// Clears n ints with a kernel (not a memset node, so it is safe inside graphs).
extern "C" int lpa_k_zero_i32(int32_t* p, int32_t n, void* stream) {
  zero_i32_kernel<<<(n + 255) / 256, 256, 0, static_cast<hipStream_t>(stream)>>>(p, n);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

// The graph of one batch, built node by node (no stream is put into capture
// mode, so other threads' device-wide calls never meet a capturing stream):
// the table copy from pinned host memory, the queue reset, the persistent fit,
// the FP64 refit and the count reduction, in that order.
namespace {
// Kernel-node arguments of a batch graph (the values the parameter arrays
// point at live here while a node is added or updated).
struct BatchNodeArgs {
  const BatchHeader* hdr;
  const LaunchK* frames;
  const int64_t* first;
  int32_t* queue;
  void* fit[4];
  void* refit[3];
  BatchNodeArgs(const BatchHeader* h, const LaunchK* f, const int64_t* fi, int32_t* q)
      : hdr(h), frames(f), first(fi), queue(q), fit{&hdr, &frames, &first, &queue}, refit{&hdr, &frames, &first} {}
};

bool batch_fit_params(BatchNodeArgs& a, int32_t src_kind, int32_t block, int32_t lds_floats2, int32_t grid,
                      hipKernelNodeParams* p) {
  *p = hipKernelNodeParams{};
  switch (src_kind) {
    case SRC_RAW_U16: p->func = reinterpret_cast<void*>(&fit_batch_kernel<SRC_RAW_U16>); break;
    case SRC_RAW_F32: p->func = reinterpret_cast<void*>(&fit_batch_kernel<SRC_RAW_F32>); break;
    case SRC_PLANE_F32: p->func = reinterpret_cast<void*>(&fit_batch_kernel<SRC_PLANE_F32>); break;
    case SRC_PLANE_F16: p->func = reinterpret_cast<void*>(&fit_batch_kernel<SRC_PLANE_F16>); break;
    default: return false;
  }
  p->gridDim = dim3(grid);
  p->blockDim = dim3(block);
  p->sharedMemBytes = (unsigned)((size_t)lds_floats2 * sizeof(float2));
  p->kernelParams = a.fit;
  return true;
}

void batch_refit_params(BatchNodeArgs& a, int32_t refit_lds_bytes, int32_t refit_grid, int32_t raw_f32,
                        hipKernelNodeParams* p) {
  *p = hipKernelNodeParams{};
  p->func = raw_f32 ? reinterpret_cast<void*>(&refit_batch_kernel<float>)
                    : reinterpret_cast<void*>(&refit_batch_kernel<uint16_t>);
  p->gridDim = dim3(refit_grid);
  p->blockDim = dim3(kRefitThreads);
  p->sharedMemBytes = (unsigned)refit_lds_bytes;
  p->kernelParams = a.refit;
}
}  // namespace

extern "C" int lpa_k_batch_graph(hipGraph_t* out, hipGraphNode_t* fit_node, hipGraphNode_t* refit_node,
                                 void* d_table, const void* h_table, size_t copy_bytes, const BatchHeader* d_hdr,
                                 const LaunchK* d_frames, const int64_t* d_first, int32_t* d_queue, int32_t src_kind,
                                 int32_t block, int32_t lds_floats2, int32_t refit_lds_bytes, int32_t grid,
                                 int32_t refit_grid, int32_t cap, int32_t raw_f32) {
  *out = nullptr;
  hipGraph_t g = nullptr;
  if (hipGraphCreate(&g, 0) != hipSuccess) return -2;
  hipGraphNode_t n_copy = nullptr, n_zero = nullptr, n_fit = nullptr, n_refit = nullptr, n_stats = nullptr;
  hipError_t e = hipGraphAddMemcpyNode1D(&n_copy, g, nullptr, 0, d_table, h_table, copy_bytes, hipMemcpyHostToDevice);
  hipKernelNodeParams p{};
  int n_q = kXcds;
  void* zero_args[] = {&d_queue, &n_q};
  p.func = reinterpret_cast<void*>(&zero_i32_kernel);
  p.gridDim = dim3(1);
  p.blockDim = dim3(64);
  p.sharedMemBytes = 0;
  p.kernelParams = zero_args;
  p.extra = nullptr;
  // plane storage: every frame's pre-pass between the table copy and the fit
  hipGraphNode_t n_first = n_copy;
  if (src_kind == SRC_PLANE_F32 || src_kind == SRC_PLANE_F16) {
    hipGraphNode_t n_pre = nullptr;
    void* pre_args[] = {&d_hdr, &d_frames};
    hipKernelNodeParams q{};
    q.func = src_kind == SRC_PLANE_F16 ? reinterpret_cast<void*>(&prepass_batch_kernel<true>)
                                       : reinterpret_cast<void*>(&prepass_batch_kernel<false>);
    q.gridDim = dim3(128, (unsigned)cap * kMaxSensors);
    q.blockDim = dim3(256);
    q.sharedMemBytes = 0;
    q.kernelParams = pre_args;
    if (e == hipSuccess) e = hipGraphAddKernelNode(&n_pre, g, &n_copy, 1, &q);
    n_first = n_pre;
  }
  if (e == hipSuccess) e = hipGraphAddKernelNode(&n_zero, g, &n_first, 1, &p);
  BatchNodeArgs args(d_hdr, d_frames, d_first, d_queue);
  if (e == hipSuccess && !batch_fit_params(args, src_kind, block, lds_floats2, grid, &p)) e = hipErrorInvalidValue;
  if (e == hipSuccess) e = hipGraphAddKernelNode(&n_fit, g, &n_zero, 1, &p);
  batch_refit_params(args, refit_lds_bytes, refit_grid, raw_f32, &p);
  if (e == hipSuccess) e = hipGraphAddKernelNode(&n_refit, g, &n_fit, 1, &p);
  void* stats_args[] = {&d_hdr, &d_frames};
  p = hipKernelNodeParams{};
  p.func = reinterpret_cast<void*>(&stats_frames_kernel);
  p.gridDim = dim3(cap);
  p.blockDim = dim3(256);
  p.sharedMemBytes = 0;
  p.kernelParams = stats_args;
  if (e == hipSuccess) e = hipGraphAddKernelNode(&n_stats, g, &n_refit, 1, &p);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    return -2;
  }
  *out = g;
  *fit_node = n_fit;
  *refit_node = n_refit;
  return 0;
}

extern "C" int lpa_k_batch_graph_set_lds(hipGraphExec_t exec, hipGraphNode_t fit_node, hipGraphNode_t refit_node,
                                         const BatchHeader* d_hdr, const LaunchK* d_frames, const int64_t* d_first,
                                         int32_t* d_queue, int32_t src_kind, int32_t block, int32_t lds_floats2,
                                         int32_t refit_lds_bytes, int32_t grid, int32_t refit_grid, int32_t raw_f32) {
  BatchNodeArgs args(d_hdr, d_frames, d_first, d_queue);
  hipKernelNodeParams p{};
  if (!batch_fit_params(args, src_kind, block, lds_floats2, grid, &p)) return -1;
  if (hipGraphExecKernelNodeSetParams(exec, fit_node, &p) != hipSuccess) return -2;
  batch_refit_params(args, refit_lds_bytes, refit_grid, raw_f32, &p);
  if (hipGraphExecKernelNodeSetParams(exec, refit_node, &p) != hipSuccess) return -2;
  return 0;
}
