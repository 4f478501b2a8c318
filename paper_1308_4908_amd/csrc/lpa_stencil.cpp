// lpa_stencil.cpp -- pre-computed window weights for translation-only rigs.
//
// The paper's GPU implementation precomputes the window weights for registered
// sensors at the output resolution (Sec. 8): when every sensor map T_s and the
// output map O are translations, the offset from output pixel (u, v) to a
// channel-c sample of sensor s is d = (k + dx_s, l + dy_s), with integer (k, l)
// of fixed parity given the pixel's parity and the sub-lattice, and
// (dx_s, dy_s) the sensor's translation minus the output map's.  So the set of
// in-window samples, their window weights K(d) and monomials are the same for
// every pixel of one parity: they are tabulated here, in FP64 and rounded once
// to FP32, per (channel, parity, radius, sensor).
//
// Each entry holds its sample's LDS offset from the output pixel's own
// position for the launch's row pitch (reg_w, part of the table's key).
//
// Support and weight follow the definition the kernels and the oracle share:
// the disc |d| < r' with K = exp(-|d|^2 / h') - exp(-r'^2 / h') > 0.  The
// monomials are taken in the launch's scaled coordinates (s d, s the radius'
// coordinate scale), like the general fit, so the solves see the same system.
#include <cmath>
#include <cstring>
#include <vector>

#include "lpa_host.hpp"

namespace lpa {
namespace {

// Hankel moment index of x^p y^q (degree-major, then by the power of y).
constexpr int hankel(int p, int q) { return (p + q) * (p + q + 1) / 2 + q; }

constexpr size_t kMaxTablesPerRig = 64;

bool is_translation(const double* a) { return a[0] == 1.0 && a[1] == 0.0 && a[3] == 0.0 && a[4] == 1.0; }

}  // namespace

lpa_status stencil_table(lpa_rig* rig, const Resolved& R, const LaunchK& K, const StencilTable** out) {
  const lpa_params& p = R.p;
  const double* O = p.out_affine;
  if (!is_translation(O))
    return set_error(LPA_ERR_UNSUPPORTED, "pre-computed weights need an output map that is a translation");
  for (int s = 0; s < rig->n; ++s)
    if (!is_translation(rig->desc[s].affine))
      return set_error(LPA_ERR_UNSUPPORTED, "pre-computed weights need translation-only sensor maps (sensor %d)", s);

  // The table depends on the output map's translation, the radii and the
  // windows (through K.sc: radius, coordinate scale per channel class).
  std::vector<double> key = {O[2], O[5], (double)p.n_scales};
  for (int s = 0; s < rig->n; ++s) key.push_back((double)K.s[s].reg_w);
  for (int m = 0; m < p.n_scales; ++m)
    for (int cls = 0; cls < 2; ++cls) {
      key.push_back(K.sc[m].radius[cls]);
      key.push_back((double)K.sc[m].coord_scale[cls]);
      key.push_back(R.h[m] * (cls == 1 ? p.green_ratio * p.green_ratio : 1.0));
    }
  std::lock_guard<std::mutex> g(rig->stencil_mu);
  for (const auto& t : rig->stencils)
    if (t.key == key) {
      *out = static_cast<const StencilTable*>(t.d);
      return LPA_OK;
    }
  if (rig->stencils.size() >= kMaxTablesPerRig)
    return set_error(LPA_ERR_UNSUPPORTED, "more than %zu pre-computed-weight parameter classes on one rig",
                     kMaxTablesPerRig);

  std::vector<StencilSeg> seg(3 * 4 * kMaxScales * kMaxSensors, StencilSeg{0, 0});
  std::vector<StencilEntry> ents;
  for (int c = 0; c < 3; ++c) {
    const int cls = c == 1 ? 1 : 0;
    const double kappa2 = cls == 1 ? p.green_ratio * p.green_ratio : 1.0;
    for (int par = 0; par < 4; ++par) {
      const int pu = par & 1, pv = par >> 1;
      for (int m = 0; m < p.n_scales; ++m) {
        const double r = K.sc[m].radius[cls];
        const double h = R.h[m] * kappa2;
        const double cs = (double)K.sc[m].coord_scale[cls];
        const double k_edge = std::exp(-r * r / h);
        for (int s = 0; s < rig->n; ++s) {
          const SensorK& S = rig->k[s];
          const SensorK& S_l = K.s[s];  // the launch's LDS region bound (row pitch)
          const double tx = rig->desc[s].affine[2] - O[2], ty = rig->desc[s].affine[5] - O[5];
          const int off = (int)ents.size();
          for (int q = 0; q < S.sub_n[c]; ++q) {
            // sample column x = u + k lies on the sub-lattice: k = ox - u (mod 2)
            const int kp = ((S.sub_ox[c][q] - pu) % 2 + 2) % 2, lp = ((S.sub_oy[c][q] - pv) % 2 + 2) % 2;
            // in-window offsets: |k + tx| < r, |l + ty| < r
            const int k0 = (int)std::floor(-tx - r) - 1, k1 = (int)std::ceil(-tx + r) + 1;
            if (!(std::fabs(tx) < 1e6 && std::fabs(ty) < 1e6))
              return set_error(LPA_ERR_UNSUPPORTED, "sensor %d is offset by more than 1e6 px from the output grid", s);
            const int l0 = (int)std::floor(-ty - r) - 1, l1 = (int)std::ceil(-ty + r) + 1;
            for (int l = l0; l <= l1; ++l) {
              if (((l - lp) & 1) != 0) continue;
              for (int k = k0; k <= k1; ++k) {
                if (((k - kp) & 1) != 0) continue;
                const double dx = k + tx, dy = l + ty;
                const double d2 = dx * dx + dy * dy;
                if (!(d2 < r * r)) continue;
                const double w = std::exp(-d2 / h) - k_edge;
                if (!(w > 0.0)) continue;
                StencilEntry e;
                std::memset(&e, 0, sizeof(e));
                const double x = dx * cs, y = dy * cs;
                double xp[5] = {1, x, x * x, x * x * x, x * x * x * x};
                double yp[5] = {1, y, y * y, y * y * y, y * y * y * y};
                for (int pp = 0; pp <= 4; ++pp)
                  for (int qq = 0; pp + qq <= 4; ++qq) e.a[hankel(pp, qq)] = (float)(w * xp[pp] * yp[qq]);
                e.delta = l * S_l.reg_w + k;
                ents.push_back(e);
              }
            }
          }
          StencilSeg& sg = seg[((c * 4 + par) * kMaxScales + m) * kMaxSensors + s];
          sg.off = off;
          sg.n = (int)ents.size() - off;
        }
      }
    }
  }

  const size_t bytes = StencilTable::entries_offset() + ents.size() * sizeof(StencilEntry);
  std::vector<char> host(bytes, 0);
  std::memcpy(host.data(), seg.data(), seg.size() * sizeof(StencilSeg));
  if (!ents.empty())
    std::memcpy(host.data() + StencilTable::entries_offset(), ents.data(), ents.size() * sizeof(StencilEntry));
  lpa_ctx* ctx = rig->ctx;
  if (ctx->used.fetch_add(bytes) + bytes > ctx->budget) {
    ctx->used.fetch_sub(bytes);
    return set_error(LPA_ERR_OOM, "HBM budget of %zu bytes exceeded", ctx->budget);
  }
  void* d = nullptr;
  hipError_t e = hipMalloc(&d, bytes);
  if (e == hipSuccess) e = hipMemcpy(d, host.data(), bytes, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    if (d) (void)hipFree(d);
    ctx->used.fetch_sub(bytes);
    return device_error(ctx, e, "pre-computed-weight table");
  }
  rig->stencils.push_back(lpa_rig::Stencil{key, d, bytes});
  *out = static_cast<const StencilTable*>(d);
  return LPA_OK;
}

void stencil_free(lpa_rig* rig) {
  std::lock_guard<std::mutex> g(rig->stencil_mu);
  for (auto& t : rig->stencils) {
    (void)hipFree(t.d);
    rig->ctx->used.fetch_sub(t.bytes);
  }
  rig->stencils.clear();
}

}  // namespace lpa
