// lpa_api.cpp -- the C ABI of include/lpa.h: contexts, rigs (with their
// resident calibration planes), argument validation, launch-descriptor
// construction and the single-frame paths (isotropic LPA, CALPA's three
// passes, pre-computed weights).  Batched and served paths live in
// lpa_batch.cpp / lpa_serve.cpp, the pre-computed-weight tables in
// lpa_stencil.cpp, the tuner in lpa_tune.cpp.
#include "lpa_host.hpp"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

namespace lpa {

thread_local char g_last_error[512] = "";

lpa_status set_error(lpa_status st, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
  va_end(ap);
  return st;
}

lpa_status device_error(lpa_ctx* ctx, hipError_t e, const char* what) {
  (void)hipGetLastError();  // leave no error state behind for the caller's own HIP calls
  const lpa_status st = set_error(LPA_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
  if (ctx) {
    // the first failure's message, for every later refusal (it may have
    // happened on the serving thread)
    std::lock_guard<std::mutex> g(ctx->fail_mu);
    if (!ctx->failed.load()) std::snprintf(ctx->fail_msg, sizeof(ctx->fail_msg), "%s", g_last_error);
    ctx->failed.store(true);
  }
  return st;
}

// Colour (0 R, 1 G, 2 B) of CFA cell [2 * row parity + column parity].
static const int kCfaTable[4][4] = {
    {0, 1, 1, 2},  // RGGB
    {2, 1, 1, 0},  // BGGR
    {1, 0, 2, 1},  // GRBG
    {1, 2, 0, 1},  // GBRG
};

static bool finite6(const double* a) {
  for (int i = 0; i < 6; ++i)
    if (!std::isfinite(a[i])) return false;
  return true;
}

lpa_status validate_rig(const lpa_rig_desc* d) {
  if (!d || !d->sensors) return set_error(LPA_ERR_INVALID_ARG, "rig descriptor is NULL");
  if (d->n_sensors < 1 || d->n_sensors > LPA_MAX_SENSORS)
    return set_error(LPA_ERR_INVALID_ARG, "n_sensors %d outside 1..%d", d->n_sensors, LPA_MAX_SENSORS);
  for (int s = 0; s < d->n_sensors; ++s) {
    const lpa_sensor_desc& S = d->sensors[s];
    if (S.width < 1 || S.height < 1 || S.width > (1 << 16) || S.height > (1 << 16))
      return set_error(LPA_ERR_INVALID_ARG, "sensor %d: size %dx%d invalid", s, S.width, S.height);
    if (S.cfa < 0 || S.cfa > 3) return set_error(LPA_ERR_INVALID_ARG, "sensor %d: cfa %d invalid", s, S.cfa);
    if (S.bit_depth < 1 || S.bit_depth > 16)
      return set_error(LPA_ERR_INVALID_ARG, "sensor %d: bit_depth %d invalid", s, S.bit_depth);
    if (!finite6(S.affine)) return set_error(LPA_ERR_INVALID_ARG, "sensor %d: affine not finite", s);
    const double det = S.affine[0] * S.affine[4] - S.affine[1] * S.affine[3];
    if (!(std::fabs(det) > 1e-12)) return set_error(LPA_ERR_INVALID_ARG, "sensor %d: affine not invertible", s);
    if (!(S.exposure > 0) || !std::isfinite(S.exposure))
      return set_error(LPA_ERR_INVALID_ARG, "sensor %d: exposure must be > 0", s);
    if (!(S.gain > 0) || !std::isfinite(S.gain)) return set_error(LPA_ERR_INVALID_ARG, "sensor %d: gain must be > 0", s);
    if (!(S.read_sigma > 0) || !std::isfinite(S.read_sigma))
      return set_error(LPA_ERR_INVALID_ARG, "sensor %d: read_sigma must be > 0", s);
    {
      // the FP32 inverse variance of a dark sample must be finite
      const double v = S.read_sigma * S.read_sigma / (S.gain * S.exposure * S.gain * S.exposure);
      if (!(v > 1e-30) || !(v < 1e30))
        return set_error(LPA_ERR_INVALID_ARG, "sensor %d: read noise variance out of FP32 range", s);
    }
    if (!std::isfinite(S.black_level) || !(S.saturation > S.black_level))
      return set_error(LPA_ERR_INVALID_ARG, "sensor %d: saturation must exceed black_level", s);
    if (S.calib) {
      const lpa_calib& C = *S.calib;
      const int64_t n = (int64_t)S.width * S.height;
      const double ge = S.gain * S.exposure;
      for (int64_t i = 0; i < n; ++i) {
        if (C.bias && !std::isfinite(C.bias[i]))
          return set_error(LPA_ERR_INVALID_ARG, "sensor %d: bias frame not finite at pixel %lld", s, (long long)i);
        const double a = C.prnu ? C.prnu[i] : 1.0;
        if (!(a > 0) || !std::isfinite(a))
          return set_error(LPA_ERR_INVALID_ARG, "sensor %d: non-uniformity must be > 0 (pixel %lld)", s, (long long)i);
        const double rv = C.read_var ? C.read_var[i] : S.read_sigma * S.read_sigma;
        const double v = rv / (ge * a * ge * a);
        if (!(rv > 0) || !std::isfinite(rv) || !(v > 1e-30) || !(v < 1e30))
          return set_error(LPA_ERR_INVALID_ARG, "sensor %d: readout variance invalid or out of FP32 range (pixel %lld)",
                           s, (long long)i);
        if (C.saturation && std::isnan(C.saturation[i]))
          return set_error(LPA_ERR_INVALID_ARG, "sensor %d: saturation frame is NaN at pixel %lld", s, (long long)i);
      }
    }
  }
  return LPA_OK;
}

// Device plane of a sensor's calibration frames: per pixel (b_i, a_i,
// Var[r_i], saturation_i), the saturation -inf where the defect mask is set.
// The frames' values are kept as given (the FP64 refit decodes with them).
static std::vector<float4> pack_calib(const lpa_sensor_desc& S) {
  const lpa_calib& C = *S.calib;
  const int64_t n = (int64_t)S.width * S.height;
  std::vector<float4> out((size_t)n);
  for (int64_t i = 0; i < n; ++i) {
    const double a = C.prnu ? C.prnu[i] : 1.0;
    float4 c;
    c.x = C.bias ? C.bias[i] : (float)S.black_level;
    c.y = (float)a;
    c.z = C.read_var ? C.read_var[i] : (float)(S.read_sigma * S.read_sigma);
    c.w = C.saturation ? C.saturation[i] : (float)S.saturation;
    if (C.defect && C.defect[i]) c.w = -INFINITY;
    out[(size_t)i] = c;
  }
  return out;
}

lpa_status resolve_params(const lpa_params* p, Resolved* r) {
  if (!p) return set_error(LPA_ERR_INVALID_ARG, "params is NULL");
  if (p->out_w < 1 || p->out_h < 1 || p->out_w > (1 << 16) || p->out_h > (1 << 16))
    return set_error(LPA_ERR_INVALID_ARG, "output size %dx%d invalid", p->out_w, p->out_h);
  if (!finite6(p->out_affine)) return set_error(LPA_ERR_INVALID_ARG, "out_affine not finite");
  if (p->order < 0 || p->order > 2) return set_error(LPA_ERR_INVALID_ARG, "order %d outside 0..2", p->order);
  if (p->n_scales < 1 || p->n_scales > LPA_MAX_SCALES)
    return set_error(LPA_ERR_INVALID_ARG, "n_scales %d outside 1..%d", p->n_scales, LPA_MAX_SCALES);
  for (int m = 0; m < p->n_scales; ++m) {
    if (!(p->radii[m] > 0) || !std::isfinite(p->radii[m]))
      return set_error(LPA_ERR_INVALID_ARG, "radius %d must be > 0", m);
    if (m > 0 && !(p->radii[m] > p->radii[m - 1]))
      return set_error(LPA_ERR_INVALID_ARG, "radii must be strictly ascending");
    if (!std::isfinite(p->h[m])) return set_error(LPA_ERR_INVALID_ARG, "h[%d] not finite", m);
  }
  if (p->n_scales > 1 && (!(p->gamma > 0) || !std::isfinite(p->gamma)))
    return set_error(LPA_ERR_INVALID_ARG, "gamma must be > 0");
  if (!(p->green_ratio > 0) || !std::isfinite(p->green_ratio))
    return set_error(LPA_ERR_INVALID_ARG, "green_ratio must be > 0");
  if (p->storage < LPA_STORE_FUSED || p->storage > LPA_STORE_FP16)
    return set_error(LPA_ERR_INVALID_ARG, "storage %d invalid", p->storage);
  if (!std::isfinite(p->tau_inv) || !std::isfinite(p->tau_fp64))
    return set_error(LPA_ERR_INVALID_ARG, "thresholds not finite");
  if (!std::isfinite(p->value_tol)) return set_error(LPA_ERR_INVALID_ARG, "value_tol not finite");
  r->p = *p;
  r->tau_inv = p->tau_inv > 0 ? p->tau_inv : 1e-5;
  r->tau_fp64 = p->tau_fp64 > 0 ? p->tau_fp64 : 1e-3;
  r->gamma = p->n_scales > 1 ? p->gamma : 1.0;
  for (int m = 0; m < p->n_scales; ++m) r->h[m] = p->h[m] > 0 ? p->h[m] : 2.0 * p->radii[m] * p->radii[m] / 9.0;
  if (p->mode != LPA_MODE_LPA && p->mode != LPA_MODE_CALPA)
    return set_error(LPA_ERR_INVALID_ARG, "mode %d invalid", p->mode);
  if (p->mode == LPA_MODE_CALPA) {
    const double vals[] = {p->alpha, p->lambda1, p->lambda2, p->grad_radius, p->grad_h, p->max_stretch};
    for (double v : vals)
      if (!std::isfinite(v)) return set_error(LPA_ERR_INVALID_ARG, "adaptive parameters not finite");
    // lambda1 > 0: with no gradient in the analysis window s1 = s2 = 0 and the
    // elongation (s1 + lambda1) / (s2 + lambda1) would be 0/0
    if (!(p->alpha >= 0) || !(p->lambda1 > 0) || !(p->lambda2 >= 0))
      return set_error(LPA_ERR_INVALID_ARG, "alpha and lambda2 must be >= 0, lambda1 > 0");
    if (p->grad_order < 0 || p->grad_order > 2)
      return set_error(LPA_ERR_INVALID_ARG, "grad_order %d invalid", p->grad_order);
    if (p->grad_halfwin < 0 || p->grad_halfwin > 16)
      return set_error(LPA_ERR_INVALID_ARG, "grad_halfwin %d invalid (0..16)", p->grad_halfwin);
    if (p->max_stretch != 0 && !(p->max_stretch >= 1 && p->max_stretch <= 8))
      return set_error(LPA_ERR_INVALID_ARG, "max_stretch %g invalid (1..8)", p->max_stretch);
    r->grad_order = p->grad_order == 0 ? 1 : p->grad_order;
    r->grad_radius = p->grad_radius > 0 ? p->grad_radius : p->radii[p->n_scales > 1 ? 1 : 0];
    r->grad_h = p->grad_h > 0 ? p->grad_h : 2.0 * r->grad_radius * r->grad_radius / 9.0;
    r->max_stretch = p->max_stretch == 0 ? 2.0 : p->max_stretch;
  }
  return LPA_OK;
}

lpa_status validate_frame(const lpa_rig* rig, const lpa_frame* f, bool need_device) {
  if (!f) return set_error(LPA_ERR_INVALID_ARG, "frame is NULL");
  if (f->n_sensors != rig->n) return set_error(LPA_ERR_INVALID_ARG, "frame has %d sensors, rig has %d", f->n_sensors, rig->n);
  if (f->dtype != LPA_DTYPE_U16 && f->dtype != LPA_DTYPE_F32) return set_error(LPA_ERR_INVALID_ARG, "dtype %d invalid", f->dtype);
  if (f->memory != LPA_MEM_DEVICE && f->memory != LPA_MEM_HOST) return set_error(LPA_ERR_INVALID_ARG, "memory %d invalid", f->memory);
  if (need_device && f->memory != LPA_MEM_DEVICE)
    return set_error(LPA_ERR_INVALID_ARG, "lpa_reconstruct needs device-resident frames");
  const int64_t es = f->dtype == LPA_DTYPE_U16 ? 2 : 4;
  for (int s = 0; s < rig->n; ++s) {
    if (!f->raw[s]) return set_error(LPA_ERR_INVALID_ARG, "raw[%d] is NULL", s);
    if (f->row_pitch_bytes[s] < es * rig->desc[s].width || f->row_pitch_bytes[s] % es)
      return set_error(LPA_ERR_INVALID_ARG, "row_pitch_bytes[%d] = %lld invalid", s, (long long)f->row_pitch_bytes[s]);
  }
  return LPA_OK;
}

lpa_status validate_output(const lpa_params* p, const lpa_output* o) {
  if (!o || !o->rgb) return set_error(LPA_ERR_INVALID_ARG, "output rgb is NULL");
  if (o->row_pitch_bytes < (int64_t)12 * p->out_w || o->row_pitch_bytes % 4)
    return set_error(LPA_ERR_INVALID_ARG, "output row pitch %lld invalid", (long long)o->row_pitch_bytes);
  if (o->scale_map && o->scale_map_pitch < (int64_t)3 * p->out_w)
    return set_error(LPA_ERR_INVALID_ARG, "scale_map pitch %lld invalid", (long long)o->scale_map_pitch);
  if (o->sd_map && (o->sd_map_pitch < (int64_t)12 * p->out_w || o->sd_map_pitch % 4))
    return set_error(LPA_ERR_INVALID_ARG, "sd_map pitch %lld invalid", (long long)o->sd_map_pitch);
  if (o->grad_map && (o->grad_map_pitch < (int64_t)8 * p->out_w || o->grad_map_pitch % 8 ||
                      reinterpret_cast<uintptr_t>(o->grad_map) % 8))
    return set_error(LPA_ERR_INVALID_ARG, "grad_map pitch %lld or alignment invalid", (long long)o->grad_map_pitch);
  if (o->steer_map && (o->steer_map_pitch < (int64_t)16 * p->out_w || o->steer_map_pitch % 16 ||
                       reinterpret_cast<uintptr_t>(o->steer_map) % 16))
    return set_error(LPA_ERR_INVALID_ARG, "steer_map pitch %lld or alignment invalid", (long long)o->steer_map_pitch);
  if ((o->grad_map || o->steer_map) && p->mode != LPA_MODE_CALPA)
    return set_error(LPA_ERR_INVALID_ARG, "grad_map and steer_map are CALPA outputs");
  return LPA_OK;
}

// Per-sensor constants that do not depend on the launch.
void rig_constants(const lpa_sensor_desc& S, SensorK* k) {
  std::memset(k, 0, sizeof(*k));
  const double* a = S.affine;
  for (int i = 0; i < 6; ++i) k->fwd[i] = a[i];
  const double det = a[0] * a[4] - a[1] * a[3];
  k->inv[0] = a[4] / det;
  k->inv[1] = -a[1] / det;
  k->inv[2] = (a[1] * a[5] - a[4] * a[2]) / det;
  k->inv[3] = -a[3] / det;
  k->inv[4] = a[0] / det;
  k->inv[5] = (a[3] * a[2] - a[0] * a[5]) / det;
  k->rownorm[0] = std::sqrt(k->inv[0] * k->inv[0] + k->inv[1] * k->inv[1]);
  k->rownorm[1] = std::sqrt(k->inv[3] * k->inv[3] + k->inv[4] * k->inv[4]);
  const double ge = S.gain * S.exposure;
  k->inv_ge = (float)(1.0 / ge);
  k->gain = (float)S.gain;
  k->read_var = (float)(S.read_sigma * S.read_sigma);
  k->black = (float)S.black_level;
  k->sat = (float)S.saturation;
  k->gain64 = S.gain;
  k->ge64 = ge;
  k->inv_ge64 = 1.0 / ge;
  k->black64 = S.black_level;
  k->read_var64 = S.read_sigma * S.read_sigma;
  k->sat64 = S.saturation;
  k->norm_decode = std::ldexp(1.0f, S.bit_depth);
  // FP16 storage offset: 2^(bits-1) makes every raw value of up to 12 bits
  // exact in FP16 (integers of magnitude <= 2048); deeper ADCs store the
  // value above the black level (exact up to 2048 DN above it)
  k->norm_offset = S.bit_depth <= 12 ? std::ldexp(1.0f, S.bit_depth - 1) : (float)S.black_level;
  k->width = S.width;
  k->height = S.height;
  for (int c = 0; c < 3; ++c) {
    int n = 0;
    for (int oy = 0; oy < 2; ++oy)
      for (int ox = 0; ox < 2; ++ox)
        if (kCfaTable[S.cfa][2 * oy + ox] == c && n < 2) {
          k->sub_ox[c][n] = (int8_t)ox;
          k->sub_oy[c][n] = (int8_t)oy;
          ++n;
        }
    k->sub_n[c] = (int8_t)n;
  }
}

// LDS the fit kernels declare statically beside the staged tile (one Region
// per sensor, 128 bytes, and the persistent kernel's tile index), rounded up:
// the staged tile and these arrays together stay within the per-workgroup
// limit.
constexpr int64_t kStaticLdsReserve = 256;

// Default accuracy target of the output values (lpa_params.value_tol = 0).
constexpr double kDefaultValueTol = 1e-4;
// |dC0| <= kRoundingFactor u S for the FP32 fit, S its rounding bound: each
// moment term goes through a few roundings (products, then the running sum);
// an FP32 emulation of the fit on the full workload's supports gave at most
// 5.5 u times the componentwise condition, which S bounds from above.
constexpr double kRoundingFactor = 8.0;
// Window weights are computed from FP32 offsets, whose rounding moves |s d|^2
// by up to about kOffsetRounding u |s d|^2 (the box origin, the steps and the
// square each round once).  The weight then moves by ln2 2^-|s d|^2 times
// that: relative to the weight this stays bounded inside the window but not
// near its edge, where the weight vanishes while 2^-|s d|^2 tends to e_edge.
// The part not proportional to the weight, up to ln2 e_edge R^2 iv per sample
// (R^2 = |s r'|^2), enters the bound as edge_coef times
// G_R (sum iv |f| + C_R sum iv) over the samples within reach, with G_R and
// C_R the sums |g_i|, |C_i| times the monomials' bound on the window.  An FP32
// emulation of the fits on 16x resampled output (few samples per window,
// order 1), where this term decides, needed a multiple of 2.
constexpr double kOffsetRounding = 4.0;

// Fill the launch-dependent parts of a descriptor.  Returns false if the
// LDS footprint of the requested tile does not fit.
lpa_status build_launch(const lpa_rig* rig, const Resolved& R, const lpa_frame* frame, const lpa_output* out,
                        int src_kind, const void* const* srcs, const int64_t* pitches, int tile_w, int tile_h,
                        LaunchK* K) {
  const lpa_params& p = R.p;
  std::memset(K, 0, sizeof(*K));
  if (tile_w < 2 || tile_h < 2 || (tile_w & 1) || (tile_h & 1) || tile_w * tile_h > 256)
    return set_error(LPA_ERR_INVALID_ARG, "tile %dx%d: sides must be even, at most 256 pixels", tile_w, tile_h);
  for (int i = 0; i < 6; ++i) K->out_affine[i] = p.out_affine[i];
  K->out_w = p.out_w;
  K->out_h = p.out_h;
  K->tile_w = tile_w;
  K->tile_h = tile_h;
  K->tiles_x = (p.out_w + tile_w - 1) / tile_w;
  K->tiles_y = (p.out_h + tile_h - 1) / tile_h;
  K->n_sensors = rig->n;
  K->n_scales = p.n_scales;
  K->order = p.order;
  K->src_kind = src_kind;
  K->gamma = (float)R.gamma;
  K->tau_inv = (float)R.tau_inv;
  K->tau_fp64 = (float)R.tau_fp64;
  K->use_fp64 = (p.flags & LPA_FLAG_NO_FP64_FALLBACK) ? 0 : 1;
  // FP64 values where the FP32 moments' rounding bound exceeds the target:
  // kRoundingFactor u S > value_tol * max(|C0|, floor), u = 2^-24.
  double ge_max = 0;
  for (int s = 0; s < rig->n; ++s) ge_max = std::max(ge_max, rig->desc[s].gain * rig->desc[s].exposure);
  K->value_floor = (float)(1.0 / ge_max);
  const double vtol = p.value_tol == 0 ? kDefaultValueTol : p.value_tol;
  K->risk_max = (vtol < 0 || !K->use_fp64) ? INFINITY : (float)(vtol / (kRoundingFactor * std::ldexp(1.0, -24)));
  K->rgb = out->rgb;
  K->rgb_pitch = out->row_pitch_bytes;
  K->map = out->scale_map;
  K->map_pitch = out->scale_map_pitch;
  K->sd = out->sd_map;
  K->sd_pitch = out->sd_map_pitch;
  K->frame_stats = out->stats;
  K->need_var = (p.n_scales > 1 || out->sd_map) ? 1 : 0;

  for (int m = 0; m < p.n_scales; ++m) {
    for (int cls = 0; cls < 2; ++cls) {
      const double kappa = cls == 1 ? p.green_ratio : 1.0;
      const double r = p.radii[m] * kappa;
      const double h = R.h[m] * kappa * kappa;
      const double cs = std::sqrt(1.4426950408889634 / h);
      K->sc[m].radius[cls] = r;
      K->sc[m].box_radius[cls] = r * R.box_stretch;
      K->sc[m].coord_scale[cls] = (float)cs;
      const double reach = (double)(float)cs * r * (1 + 1e-4);
      K->sc[m].reach2[cls] = (float)(reach * reach);
      K->sc[m].e_edge[cls] = (float)std::exp(-r * r / h);
      K->sc[m].h[cls] = h;
      K->sc[m].edge_coef[cls] = (float)(kOffsetRounding * std::log(2.0) * std::exp(-r * r / h) * (cs * r) * (cs * r) /
                                        kRoundingFactor);
      K->sc[m].mono_r[cls] = (float)(cs * r * (1 + 1e-4));
    }
  }
  int lds = 0;
  const double* O = p.out_affine;  // output map
  for (int s = 0; s < rig->n; ++s) {
    SensorK& S = K->s[s];
    S = rig->k[s];
    S.src = srcs[s];
    S.pitch = pitches[s];
    S.raw = frame->raw[s];
    S.raw_pitch = frame->row_pitch_bytes[s];
    S.raw_f32 = frame->dtype == LPA_DTYPE_F32 ? 1 : 0;
    double wmx = 0, wmy = 0;
    for (int cls = 0; cls < 2; ++cls) {
      for (int m = 0; m < p.n_scales; ++m) {
        const double wx = K->sc[m].box_radius[cls] * S.rownorm[0];
        const double wy = K->sc[m].box_radius[cls] * S.rownorm[1];
        const double nx = std::max(1.0, std::ceil(wx - 1e-9));
        const double ny = std::max(1.0, std::ceil(wy - 1e-9));
        if (nx > 120 || ny > 120)
          return set_error(LPA_ERR_UNSUPPORTED, "window radius %g spans more than 240 sensor pixels",
                           K->sc[m].radius[cls]);
        S.nbox[cls][m][0] = (int8_t)nx;
        S.nbox[cls][m][1] = (int8_t)ny;
        wmx = std::max(wmx, wx);
        wmy = std::max(wmy, wy);
      }
    }
    S.wmax[0] = wmx;
    S.wmax[1] = wmy;
    // Every output pixel lies in the hull of the grid's corners; their sensor
    // coordinates must stay well inside int range for the kernels' indexing.
    for (int c = 0; c < 4; ++c) {
      const double u = (c & 1) ? p.out_w - 1 : 0, v = (c & 2) ? p.out_h - 1 : 0;
      const double X = O[0] * u + O[1] * v + O[2], Y = O[3] * u + O[4] * v + O[5];
      const double px = S.inv[0] * X + S.inv[1] * Y + S.inv[2];
      const double py = S.inv[3] * X + S.inv[4] * Y + S.inv[5];
      if (!(std::fabs(px) < 1e8) || !(std::fabs(py) < 1e8))
        return set_error(LPA_ERR_INVALID_ARG, "output grid maps %g px away from sensor %d", std::fmax(std::fabs(px), std::fabs(py)), s);
    }
    const double L00 = S.inv[0] * O[0] + S.inv[1] * O[3], L01 = S.inv[0] * O[1] + S.inv[1] * O[4];
    const double L10 = S.inv[3] * O[0] + S.inv[4] * O[3], L11 = S.inv[3] * O[1] + S.inv[4] * O[4];
    const double ex = std::fabs(L00) * (tile_w - 1) + std::fabs(L01) * (tile_h - 1);
    const double ey = std::fabs(L10) * (tile_w - 1) + std::fabs(L11) * (tile_h - 1);
    S.reg_w = (int)std::ceil(ex + 2 * wmx) + 8;
    S.reg_h = (int)std::ceil(ey + 2 * wmy) + 8;
    S.lds_off = lds;
    lds += S.reg_w * S.reg_h;
    if ((int64_t)lds * 8 + kStaticLdsReserve > lpa_k_fit_max_lds_bytes())
      return set_error(LPA_ERR_UNSUPPORTED, "tile %dx%d needs more than %d bytes of LDS", tile_w, tile_h,
                       lpa_k_fit_max_lds_bytes());
  }
  K->lds_floats2 = lds;
  // FP64 refit blocks: the largest whose sensors' raw footprints (the block's
  // corners widened as the kernel widens them) fit the refit launch's LDS
  static const int kRefitBlocks[][2] = {{32, 32}, {32, 16}, {16, 16}, {16, 8}, {8, 8}, {8, 4}, {4, 4}, {2, 2}};
  const int64_t es = frame->dtype == LPA_DTYPE_F32 ? 4 : 2;
  K->refit_bw = K->refit_bh = 0;
  for (const auto& b : kRefitBlocks) {
    int64_t n = 0;
    for (int s = 0; s < rig->n; ++s) {
      const SensorK& S = K->s[s];
      const double L00 = S.inv[0] * O[0] + S.inv[1] * O[3], L01 = S.inv[0] * O[1] + S.inv[1] * O[4];
      const double L10 = S.inv[3] * O[0] + S.inv[4] * O[3], L11 = S.inv[3] * O[1] + S.inv[4] * O[4];
      const double ex = std::fabs(L00) * (b[0] - 1) + std::fabs(L01) * (b[1] - 1);
      const double ey = std::fabs(L10) * (b[0] - 1) + std::fabs(L11) * (b[1] - 1);
      n += (int64_t)(std::ceil(ex + 2 * S.wmax[0]) + 8) * (int64_t)(std::ceil(ey + 2 * S.wmax[1]) + 8);
    }
    if (n * es <= lpa_k_refit_max_lds_bytes()) {
      K->refit_bw = b[0];
      K->refit_bh = b[1];
      K->refit_lds = (int32_t)n;
      break;
    }
  }
  if (!K->refit_bw) return set_error(LPA_ERR_UNSUPPORTED, "the FP64 refit cannot stage these windows");
  return LPA_OK;
}

// Tile shapes tried in order (largest first) when a tile's LDS does not fit.
static const int kTileShapes[][2] = {{16, 16}, {16, 8}, {8, 8}, {8, 4}, {4, 4}};

lpa_status build_launch_fit(const lpa_rig* rig, const Resolved& R, const lpa_frame* frame, const lpa_output* out,
                            int src_kind, const void* const* srcs, const int64_t* pitches, int pref_w, int pref_h,
                            LaunchK* K) {
  lpa_status st = build_launch(rig, R, frame, out, src_kind, srcs, pitches, pref_w, pref_h, K);
  if (st != LPA_ERR_UNSUPPORTED) return st;
  for (const auto& t : kTileShapes) {
    if (t[0] * t[1] >= pref_w * pref_h) continue;
    st = build_launch(rig, R, frame, out, src_kind, srcs, pitches, t[0], t[1], K);
    if (st != LPA_ERR_UNSUPPORTED) return st;
  }
  return st;
}

lpa_status check_ctx(lpa_ctx* ctx) {
  if (!ctx) return set_error(LPA_ERR_INVALID_ARG, "context is NULL");
  if (ctx->failed.load()) {
    std::lock_guard<std::mutex> g(ctx->fail_mu);
    return set_error(LPA_ERR_DEVICE, "context failed after an earlier device error (%s)", ctx->fail_msg);
  }
  return LPA_OK;
}

// Scratch planes for the pre-pass forms, stream-ordered (hipMallocAsync).
lpa_status alloc_async(lpa_ctx* ctx, size_t bytes, hipStream_t st, void** p, bool charge) {
  if (charge) {
    size_t used = ctx->used.fetch_add(bytes) + bytes;
    if (used > ctx->budget) {
      ctx->used.fetch_sub(bytes);
      return set_error(LPA_ERR_OOM, "HBM budget of %zu bytes exceeded", ctx->budget);
    }
  }
  hipError_t e = hipMallocAsync(p, bytes, st);
  if (e != hipSuccess) {
    if (charge) ctx->used.fetch_sub(bytes);
    *p = nullptr;
    (void)hipGetLastError();
    return set_error(LPA_ERR_OOM, "hipMallocAsync(%zu): %s", bytes, hipGetErrorString(e));
  }
  return LPA_OK;
}

void free_async(lpa_ctx* ctx, void* p, size_t bytes, hipStream_t st, bool charge) {
  if (!p) return;
  (void)hipFreeAsync(p, st);
  if (charge) ctx->used.fetch_sub(bytes);
}

// Pre-pass every sensor into planes; fills srcs/pitches and the allocations.
lpa_status run_prepass(lpa_rig* rig, const lpa_frame* f, bool to_f16, hipStream_t st, void** planes,
                       size_t* plane_bytes, const void** srcs, int64_t* pitches, bool charge) {
  lpa_ctx* ctx = rig->ctx;
  for (int s = 0; s < rig->n; ++s) {
    const SensorK& S = rig->k[s];
    const int64_t pitch = ((int64_t)S.width * (to_f16 ? 2 : 8) + 255) / 256 * 256;
    plane_bytes[s] = (size_t)pitch * S.height;
    lpa_status rs = alloc_async(ctx, plane_bytes[s], st, &planes[s], charge);
    if (rs != LPA_OK) return rs;
    const float enc = std::ldexp(1.0f, -rig->desc[s].bit_depth);
    if (lpa_k_prepass(&S, f->dtype == LPA_DTYPE_F32, f->raw[s], f->row_pitch_bytes[s], planes[s], pitch,
                                to_f16 ? 1 : 0, enc, st) != 0)
      return device_error(ctx, hipGetLastError(), "pre-pass launch");
    srcs[s] = planes[s];
    pitches[s] = pitch;
  }
  return LPA_OK;
}

// Per-tile count buffer for a frame whose output asks for the FP64-valued and
// no-data counts (lpa_output.stats); stats_end sums it into the caller's
// counters after the fit and frees it.
static lpa_status stats_begin(lpa_ctx* ctx, const lpa_output* out, LaunchK* K, hipStream_t hs, void** buf,
                              size_t* bytes) {
  *buf = nullptr;
  *bytes = 0;
  if (!out->stats) return LPA_OK;
  *bytes = (size_t)K->tiles_x * K->tiles_y * 2 * sizeof(uint32_t);
  lpa_status st = alloc_async(ctx, *bytes, hs, buf);
  if (st == LPA_OK) K->tile_stats = static_cast<uint32_t*>(*buf);
  return st;
}

static lpa_status stats_end(lpa_ctx* ctx, const lpa_output* out, const LaunchK& K, hipStream_t hs, void* buf,
                            size_t bytes, lpa_status st) {
  if (st == LPA_OK && buf &&
      lpa_k_stats_sum(K.tile_stats, (int64_t)K.tiles_x * K.tiles_y, out->stats, hs) != 0)
    st = device_error(ctx, hipGetLastError(), "count reduction");
  free_async(ctx, buf, bytes, hs);
  return st;
}

// The FP64 refit of the outputs a fit marks: a map of marks (3 bytes per
// output pixel, stream-ordered scratch) that the fit writes and refit_end's
// launch reads.  Launches whose accuracy target is off need neither.
static lpa_status refit_begin(lpa_ctx* ctx, LaunchK* K, hipStream_t hs, void** buf, size_t* bytes) {
  *buf = nullptr;
  *bytes = 0;
  if (!std::isfinite(K->risk_max)) return LPA_OK;
  *bytes = (size_t)K->out_w * K->out_h * 3;
  lpa_status st = alloc_async(ctx, *bytes, hs, buf);
  if (st == LPA_OK) {
    K->refit_map = static_cast<uint8_t*>(*buf);
    K->refit_pitch = (int64_t)3 * K->out_w;
  }
  return st;
}

static lpa_status refit_end(lpa_ctx* ctx, const LaunchK& K, hipStream_t hs, void* buf, size_t bytes,
                            lpa_status st) {
  if (st == LPA_OK && buf && lpa_k_refit(&K, hs) != 0) st = device_error(ctx, hipGetLastError(), "refit launch");
  free_async(ctx, buf, bytes, hs);
  return st;
}

// Adaptive anisotropic LPA with colour-channel correlation (Sec. 5.4, 5.5):
// gradient pass (G channel, isotropic), steering pass, steered fit of R, G, B.
// Every descriptor is built and checked before anything is enqueued.
static lpa_status calpa_impl(lpa_rig* rig, const lpa_frame* frame, const Resolved& R, const lpa_output* out,
                             hipStream_t hs, bool plain) {
  lpa_ctx* ctx = rig->ctx;
  const int storage = plain ? LPA_STORE_FP32 : R.p.storage;
  int src_kind;
  const void* srcs[LPA_MAX_SENSORS];
  int64_t pitches[LPA_MAX_SENSORS];
  void* planes[LPA_MAX_SENSORS] = {nullptr};
  size_t plane_bytes[LPA_MAX_SENSORS] = {0};
  if (storage == LPA_STORE_FUSED) {
    src_kind = frame->dtype == LPA_DTYPE_U16 ? SRC_RAW_U16 : SRC_RAW_F32;
    for (int s = 0; s < rig->n; ++s) {
      srcs[s] = frame->raw[s];
      pitches[s] = frame->row_pitch_bytes[s];
    }
  } else {
    src_kind = storage == LPA_STORE_FP16 ? SRC_PLANE_F16 : SRC_PLANE_F32;
    for (int s = 0; s < rig->n; ++s) {
      srcs[s] = nullptr;
      pitches[s] = 0;
    }
  }
  // gradient pass: one isotropic radius, order grad_order, no variance
  Resolved Rg = R;
  Rg.p.order = R.grad_order;
  Rg.p.n_scales = 1;
  Rg.p.radii[0] = R.grad_radius;
  Rg.p.h[0] = R.grad_h;
  Rg.h[0] = R.grad_h;
  Rg.box_stretch = 1;
  lpa_output og{};
  og.rgb = out->rgb;
  og.row_pitch_bytes = out->row_pitch_bytes;
  LaunchK Kg, Ks;
  lpa_status st = build_launch_fit(rig, Rg, frame, &og, src_kind, srcs, pitches, 16, 16, &Kg);
  if (st != LPA_OK) return st;
  // steered fit: boxes cover the ellipse, within max_stretch * r of the pixel
  Resolved Rs = R;
  Rs.box_stretch = R.max_stretch;
  if ((st = build_launch_fit(rig, Rs, frame, out, src_kind, srcs, pitches, 16, 16, &Ks)) != LPA_OK) return st;

  const int W = R.p.out_w, H = R.p.out_h;
  void* gbuf = nullptr;
  void* sbuf = nullptr;
  const size_t gbytes = (size_t)W * H * 8, sbytes = (size_t)W * H * 16;
  float* gptr = out->grad_map;
  int64_t gpitch = out->grad_map_pitch;
  float* sptr = out->steer_map;
  int64_t spitch = out->steer_map_pitch;
  if (!gptr) {
    if ((st = alloc_async(ctx, gbytes, hs, &gbuf)) != LPA_OK) return st;
    gptr = static_cast<float*>(gbuf);
    gpitch = (int64_t)W * 8;
  }
  if (!sptr) {
    if ((st = alloc_async(ctx, sbytes, hs, &sbuf)) != LPA_OK) {
      free_async(ctx, gbuf, gbytes, hs);
      return st;
    }
    sptr = static_cast<float*>(sbuf);
    spitch = (int64_t)W * 16;
  }
  if (storage != LPA_STORE_FUSED) {
    st = run_prepass(rig, frame, storage == LPA_STORE_FP16, hs, planes, plane_bytes, srcs, pitches);
    if (st == LPA_OK)
      for (int s = 0; s < rig->n; ++s) {
        Kg.s[s].src = Ks.s[s].src = srcs[s];
        Kg.s[s].pitch = Ks.s[s].pitch = pitches[s];
      }
  }
  Kg.grad = gptr;
  Kg.grad_pitch = gpitch;
  Kg.map = nullptr;
  Kg.sd = nullptr;
  Kg.need_var = 0;
  if (st == LPA_OK && lpa_k_grad(&Kg, hs) != 0) st = device_error(ctx, hipGetLastError(), "gradient launch");
  if (st == LPA_OK) {
    SteerArgs A{};
    A.grad = gptr;
    A.grad_pitch = gpitch;
    A.steer = sptr;
    A.steer_pitch = spitch;
    A.out_w = W;
    A.out_h = H;
    A.q = R.p.grad_halfwin;
    A.alpha = R.p.alpha;
    A.lambda1 = R.p.lambda1;
    A.lambda2 = R.p.lambda2;
    A.lo = 1.0 / (R.max_stretch * R.max_stretch);
    A.hi = R.max_stretch * R.max_stretch;
    if (lpa_k_steer(&A, hs) != 0) st = device_error(ctx, hipGetLastError(), "steering launch");
  }
  Ks.steer = sptr;
  Ks.steer_pitch = spitch;
  void* cbuf = nullptr;
  void* rbuf = nullptr;
  size_t cbytes = 0, rbytes = 0;
  if (st == LPA_OK) st = stats_begin(ctx, out, &Ks, hs, &cbuf, &cbytes);
  if (st == LPA_OK) st = refit_begin(ctx, &Ks, hs, &rbuf, &rbytes);
  KernelBracket kb(ctx, hs);
  if (st == LPA_OK) kb.mark(0);
  if (st == LPA_OK && lpa_k_fit_steered(&Ks, hs) != 0) st = device_error(ctx, hipGetLastError(), "steered fit launch");
  if (st == LPA_OK) kb.mark(1);
  st = refit_end(ctx, Ks, hs, rbuf, rbytes, st);
  if (st == LPA_OK) {
    if (rbuf) kb.mark(2);
    kb.commit(rbuf != nullptr);
  }
  st = stats_end(ctx, out, Ks, hs, cbuf, cbytes, st);
  for (int s = 0; s < rig->n; ++s) free_async(ctx, planes[s], plane_bytes[s], hs);
  free_async(ctx, gbuf, gbytes, hs);
  free_async(ctx, sbuf, sbytes, hs);
  return st;
}

KernelBracket::KernelBracket(lpa_ctx* ctx, hipStream_t hs) : ctx_(ctx), hs_(hs) {
  {
    std::lock_guard<std::mutex> g(ctx->timing_mu);
    on_ = ctx->timing;
  }
  if (!on_) return;
  for (auto& e : ev_)
    if (hipEventCreate(&e) != hipSuccess) {
      e = nullptr;
      on_ = false;
    }
}

KernelBracket::~KernelBracket() {
  for (auto& e : ev_)
    if (e) (void)hipEventDestroy(e);
}

void KernelBracket::mark(int i) {
  if (on_ && hipEventRecord(ev_[i], hs_) != hipSuccess) on_ = false;
}

void KernelBracket::commit(bool refit_launched) {
  if (!on_) return;
  on_ = false;
  if (!refit_launched) {
    (void)hipEventDestroy(ev_[2]);
    ev_[2] = nullptr;
  }
  std::lock_guard<std::mutex> g(ctx_->timing_mu);
  if (!ctx_->timing) return;  // switched off meanwhile: the destructor frees the events
  ctx_->timing_events.push_back(ev_);
  ev_ = {};
}

void timing_clear_locked(lpa_ctx* ctx) {
  for (auto& f : ctx->timing_events)
    for (auto& e : f)
      if (e) (void)hipEventDestroy(e);
  ctx->timing_events.clear();
}

// Register budget of the pre-computed-weight kernel (waves per SIMD; 0 = 3).
// Its entry loop waits on scalar loads and the LDS reads they address: 4
// waves hide more of that latency than the few spilled registers cost.
constexpr int kStencilOccupancy = 4;

lpa_status reconstruct_impl(lpa_rig* rig, const lpa_frame* frame, const lpa_params* params,
                            const lpa_output* out, void* stream, bool plain) {
  if (!rig) return set_error(LPA_ERR_INVALID_ARG, "rig is NULL");
  lpa_ctx* ctx = rig->ctx;
  lpa_status st = check_ctx(ctx);
  if (st != LPA_OK) return st;
  Resolved R;
  if ((st = resolve_params(params, &R)) != LPA_OK) return st;
  if ((st = validate_frame(rig, frame, true)) != LPA_OK) return st;
  if ((st = validate_output(params, out)) != LPA_OK) return st;
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return device_error(ctx, e, "hipSetDevice");
  hipStream_t hs = static_cast<hipStream_t>(stream);
  const bool stencil = (R.p.flags & LPA_FLAG_PRECOMPUTED_WEIGHTS) != 0;
  if (stencil && R.p.mode != LPA_MODE_LPA)
    return set_error(LPA_ERR_UNSUPPORTED, "pre-computed weights apply to isotropic windows (mode LPA)");
  if (R.p.mode == LPA_MODE_CALPA) return calpa_impl(rig, frame, R, out, hs, plain);

  const int storage = plain ? LPA_STORE_FP32 : R.p.storage;
  int src_kind;
  const void* srcs[LPA_MAX_SENSORS];
  int64_t pitches[LPA_MAX_SENSORS];
  void* planes[LPA_MAX_SENSORS] = {nullptr};
  size_t plane_bytes[LPA_MAX_SENSORS] = {0};
  int tw = 16, th = 16;

  // Descriptor first: its validation must not leave work enqueued.
  if (storage == LPA_STORE_FUSED) {
    src_kind = frame->dtype == LPA_DTYPE_U16 ? SRC_RAW_U16 : SRC_RAW_F32;
    for (int s = 0; s < rig->n; ++s) {
      srcs[s] = frame->raw[s];
      pitches[s] = frame->row_pitch_bytes[s];
    }
  } else {
    src_kind = storage == LPA_STORE_FP16 ? SRC_PLANE_F16 : SRC_PLANE_F32;
    for (int s = 0; s < rig->n; ++s) {
      srcs[s] = nullptr;
      pitches[s] = 0;
    }
  }
  TuneChoice tc;
  if (!plain && !stencil) {
    tc = ctx->tuner.choose(Tuner::key_of(rig, R, src_kind));
    tw = tc.tile_w;
    th = tc.tile_h;
  }
  LaunchK K;
  // The pre-computed-weight kernel needs one parity class per wave: 16 x 16.
  // The other forms fall back to smaller tiles when wide windows over many
  // sensors overflow the LDS of the preferred one (16 x 16 for the plain form).
  st = stencil ? build_launch(rig, R, frame, out, src_kind, srcs, pitches, 16, 16, &K)
               : build_launch_fit(rig, R, frame, out, src_kind, srcs, pitches, tw, th, &K);
  if (st != LPA_OK) return st;
  K.occupancy = tc.occupancy;
  if (stencil) {
    if ((st = stencil_table(rig, R, K, &K.stencil)) != LPA_OK) return st;
    K.occupancy = kStencilOccupancy;
  }

  if (storage != LPA_STORE_FUSED) {
    st = run_prepass(rig, frame, storage == LPA_STORE_FP16, hs, planes, plane_bytes, srcs, pitches);
    if (st == LPA_OK)
      for (int s = 0; s < rig->n; ++s) {
        K.s[s].src = srcs[s];
        K.s[s].pitch = pitches[s];
      }
  }
  void* cbuf = nullptr;
  void* rbuf = nullptr;
  size_t cbytes = 0, rbytes = 0;
  if (st == LPA_OK) st = stats_begin(ctx, out, &K, hs, &cbuf, &cbytes);
  if (st == LPA_OK) st = refit_begin(ctx, &K, hs, &rbuf, &rbytes);
  KernelBracket kb(ctx, hs);
  if (st == LPA_OK) kb.mark(0);
  if (st == LPA_OK && (stencil ? lpa_k_fit_stencil(&K, hs) : lpa_k_fit(&K, hs)) != 0)
    st = device_error(ctx, hipGetLastError(), "fit launch");
  if (st == LPA_OK) kb.mark(1);
  st = refit_end(ctx, K, hs, rbuf, rbytes, st);
  if (st == LPA_OK) {
    if (rbuf) kb.mark(2);
    kb.commit(rbuf != nullptr);
  }
  st = stats_end(ctx, out, K, hs, cbuf, cbytes, st);
  for (int s = 0; s < rig->n; ++s) free_async(ctx, planes[s], plane_bytes[s], hs);
  return st;
}

// Temporal LPA: the launch's sensors are the rig's sensors at each frame,
// sensor t * n + s being sensor s at time -t, every one with its own staged
// region and its frame's temporal factor per radius.
static lpa_status temporal_impl(lpa_rig* rig, const lpa_frame* frames, int32_t n_times, const lpa_params* params,
                                const lpa_output* out, void* stream) {
  if (!rig) return set_error(LPA_ERR_INVALID_ARG, "rig is NULL");
  lpa_ctx* ctx = rig->ctx;
  lpa_status st = check_ctx(ctx);
  if (st != LPA_OK) return st;
  if (!frames) return set_error(LPA_ERR_INVALID_ARG, "frames is NULL");
  Resolved R;
  if ((st = resolve_params(params, &R)) != LPA_OK) return st;
  if (n_times < 1) return set_error(LPA_ERR_INVALID_ARG, "n_times %d < 1", n_times);
  if ((int64_t)n_times * rig->n > LPA_MAX_SENSORS)
    return set_error(LPA_ERR_UNSUPPORTED, "%d frames of %d sensors exceed %d staged sensors", n_times, rig->n,
                     LPA_MAX_SENSORS);
  if (R.p.mode != LPA_MODE_LPA || (R.p.flags & LPA_FLAG_PRECOMPUTED_WEIGHTS))
    return set_error(LPA_ERR_UNSUPPORTED, "temporal LPA takes mode LPA without pre-computed weights");
  if (R.p.storage != LPA_STORE_FUSED)
    return set_error(LPA_ERR_UNSUPPORTED, "temporal LPA reads raw frames (storage FUSED)");
  for (int t = 0; t < n_times; ++t) {
    if ((st = validate_frame(rig, &frames[t], true)) != LPA_OK) return st;
    if (frames[t].dtype != frames[0].dtype) return set_error(LPA_ERR_INVALID_ARG, "frames of different dtypes");
  }
  if ((st = validate_output(params, out)) != LPA_OK) return st;
  const double ht_min = (double)(n_times - 1) * (n_times - 1) / 16.0;
  for (int m = 0; m < R.p.n_scales; ++m) {
    const double h = R.p.h_t[m];
    if (!(h >= 0.0) || !std::isfinite(h) || (n_times > 1 && h > 0.0 && h < ht_min))
      return set_error(LPA_ERR_INVALID_ARG, "h_t[%d] = %g: 0 or at least (n_times - 1)^2 / 16 = %g", m, h, ht_min);
  }
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return device_error(ctx, e, "hipSetDevice");
  hipStream_t hs = static_cast<hipStream_t>(stream);

  std::unique_ptr<lpa_rig> vr(new (std::nothrow) lpa_rig());
  if (!vr) return set_error(LPA_ERR_OOM, "host allocation failed");
  vr->ctx = ctx;
  vr->n = n_times * rig->n;
  lpa_frame vf{};
  vf.n_sensors = vr->n;
  vf.dtype = frames[0].dtype;
  vf.memory = LPA_MEM_DEVICE;
  const void* srcs[LPA_MAX_SENSORS];
  int64_t pitches[LPA_MAX_SENSORS];
  for (int t = 0; t < n_times; ++t)
    for (int s = 0; s < rig->n; ++s) {
      const int v = t * rig->n + s;
      vr->desc[v] = rig->desc[s];
      vr->k[v] = rig->k[s];
      vf.raw[v] = srcs[v] = frames[t].raw[s];
      vf.row_pitch_bytes[v] = pitches[v] = frames[t].row_pitch_bytes[s];
    }
  const int src_kind = vf.dtype == LPA_DTYPE_U16 ? SRC_RAW_U16 : SRC_RAW_F32;
  LaunchK K;
  if ((st = build_launch_fit(vr.get(), R, &vf, out, src_kind, srcs, pitches, 16, 16, &K)) != LPA_OK) return st;
  for (int v = 0; v < vr->n; ++v) {
    const int t = v / rig->n;
    K.s[v].time = t;
    for (int m = 0; m < R.p.n_scales; ++m)
      K.s[v].kt[m] = t == 0 ? 1.f : (R.p.h_t[m] > 0.0 ? (float)std::exp(-(double)t * t / R.p.h_t[m]) : 0.f);
  }
  for (int m = 0; m < R.p.n_scales; ++m) K.sc[m].inv_ht = R.p.h_t[m] > 0.0 ? 1.0 / R.p.h_t[m] : 0.0;
  K.occupancy = 0;

  void* cbuf = nullptr;
  void* rbuf = nullptr;
  size_t cbytes = 0, rbytes = 0;
  st = stats_begin(ctx, out, &K, hs, &cbuf, &cbytes);
  if (st == LPA_OK) st = refit_begin(ctx, &K, hs, &rbuf, &rbytes);
  KernelBracket kb(ctx, hs);
  if (st == LPA_OK) kb.mark(0);
  if (st == LPA_OK && lpa_k_fit_temporal(&K, hs) != 0) st = device_error(ctx, hipGetLastError(), "temporal fit launch");
  if (st == LPA_OK) kb.mark(1);
  st = refit_end(ctx, K, hs, rbuf, rbytes, st);
  if (st == LPA_OK) {
    if (rbuf) kb.mark(2);
    kb.commit(rbuf != nullptr);
  }
  return stats_end(ctx, out, K, hs, cbuf, cbytes, st);
}

}  // namespace lpa

using namespace lpa;

extern "C" {

lpa_status lpa_reconstruct_temporal(lpa_rig* rig, const lpa_frame* frames, int32_t n_times,
                                    const lpa_params* params, const lpa_output* out, void* hip_stream) {
  try {
    return temporal_impl(rig, frames, n_times, params, out, hip_stream);
  } catch (...) {
    return set_error(LPA_ERR_INTERNAL, "unexpected host exception");
  }
}

const char* lpa_last_error(void) { return g_last_error; }

lpa_status lpa_set_kernel_timing(lpa_ctx* ctx, int32_t on) {
  lpa_status st = check_ctx(ctx);
  if (st != LPA_OK) return st;
  std::lock_guard<std::mutex> g(ctx->timing_mu);
  timing_clear_locked(ctx);
  ctx->timing = on != 0;
  return LPA_OK;
}

lpa_status lpa_kernel_times(lpa_ctx* ctx, lpa_kernel_time* out) {
  if (!out) return set_error(LPA_ERR_INVALID_ARG, "out is NULL");
  lpa_status st = check_ctx(ctx);
  if (st != LPA_OK) return st;
  std::vector<std::array<hipEvent_t, 3>> evs;
  {
    std::lock_guard<std::mutex> g(ctx->timing_mu);
    evs.swap(ctx->timing_events);
  }
  *out = lpa_kernel_time{};
  hipError_t e = hipSetDevice(ctx->device);
  for (auto& f : evs) {
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventSynchronize(f[2] ? f[2] : f[1]);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, f[0], f[1]);
    if (e == hipSuccess) {
      out->fit_ms += ms;
      out->n_fit += 1;
    }
    if (e == hipSuccess && f[2]) {
      e = hipEventElapsedTime(&ms, f[1], f[2]);
      if (e == hipSuccess) {
        out->refit_ms += ms;
        out->n_refit += 1;
      }
    }
    for (auto& x : f)
      if (x) (void)hipEventDestroy(x);
  }
  if (e != hipSuccess) return device_error(ctx, e, "kernel timing events");
  return LPA_OK;
}

lpa_status lpa_create_ctx(int device, size_t hbm_budget_bytes, lpa_ctx** out) {
  if (!out) return set_error(LPA_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || n == 0) return set_error(LPA_ERR_DEVICE, "no HIP device: %s", hipGetErrorString(e));
  if (device < 0 || device >= n) return set_error(LPA_ERR_INVALID_ARG, "device %d outside 0..%d", device, n - 1);
  if ((e = hipSetDevice(device)) != hipSuccess) return set_error(LPA_ERR_DEVICE, "hipSetDevice: %s", hipGetErrorString(e));
  lpa_ctx* ctx = new (std::nothrow) lpa_ctx();
  if (!ctx) return set_error(LPA_ERR_OOM, "host allocation failed");
  ctx->device = device;
  hipDeviceProp_t prop;
  if ((e = hipGetDeviceProperties(&prop, device)) != hipSuccess) {
    delete ctx;
    return set_error(LPA_ERR_DEVICE, "hipGetDeviceProperties: %s", hipGetErrorString(e));
  }
  ctx->n_cu = prop.multiProcessorCount;
  size_t free_b = 0, total_b = 0;
  (void)hipMemGetInfo(&free_b, &total_b);
  ctx->budget = hbm_budget_bytes ? hbm_budget_bytes : (size_t)(0.9 * (double)free_b);
  lpa_status st = noalloc_init_device(device);
  if (st == LPA_OK) st = ctx_init_runtime(ctx);
  if (st != LPA_OK) {
    delete ctx;
    return st;
  }
  *out = ctx;
  return LPA_OK;
}

static void rig_free(lpa_rig* rig) {
  (void)hipSetDevice(rig->ctx->device);
  if (rig->d_k) (void)hipFree(rig->d_k);
  for (int s = 0; s < rig->n; ++s) {
    if (rig->k[s].calib) (void)hipFree(const_cast<float4*>(rig->k[s].calib));
    rig->ctx->used.fetch_sub(rig->calib_bytes[s]);
  }
  stencil_free(rig);
  delete rig;
}

lpa_status lpa_destroy_ctx(lpa_ctx* ctx) {
  if (!ctx) return set_error(LPA_ERR_INVALID_ARG, "context is NULL");
  ctx_shutdown_runtime(ctx);
  // rigs still alive are destroyed with their context
  std::vector<lpa_rig*> rigs;
  {
    std::lock_guard<std::mutex> g(ctx->rigs_mu);
    rigs.assign(ctx->rigs.begin(), ctx->rigs.end());
    ctx->rigs.clear();
  }
  for (lpa_rig* r : rigs) rig_free(r);
  {
    std::lock_guard<std::mutex> g(ctx->timing_mu);
    timing_clear_locked(ctx);
  }
  (void)hipGetLastError();
  delete ctx;
  return LPA_OK;
}

lpa_status lpa_create_rig(lpa_ctx* ctx, const lpa_rig_desc* desc, lpa_rig** out) {
  lpa_status st = check_ctx(ctx);
  if (st != LPA_OK) return st;
  if (!out) return set_error(LPA_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if ((st = validate_rig(desc)) != LPA_OK) return st;
  lpa_rig* rig = new (std::nothrow) lpa_rig();
  if (!rig) return set_error(LPA_ERR_OOM, "host allocation failed");
  rig->ctx = ctx;
  rig->n = desc->n_sensors;
  for (int s = 0; s < rig->n; ++s) {
    rig->desc[s] = desc->sensors[s];
    rig->desc[s].calib = nullptr;  // the frames are copied below; the caller's pointers are not kept
    rig_constants(rig->desc[s], &rig->k[s]);
  }
  hipError_t e = hipSetDevice(ctx->device);
  // Per-pixel calibration planes, resident until the rig is destroyed.
  for (int s = 0; s < rig->n && e == hipSuccess; ++s) {
    if (!desc->sensors[s].calib) continue;
    const std::vector<float4> plane = pack_calib(desc->sensors[s]);
    const size_t bytes = plane.size() * sizeof(float4);
    if (ctx->used.fetch_add(bytes) + bytes > ctx->budget) {
      ctx->used.fetch_sub(bytes);
      rig_free(rig);
      return set_error(LPA_ERR_OOM, "HBM budget of %zu bytes exceeded by calibration frames", ctx->budget);
    }
    rig->calib_bytes[s] = bytes;
    void* d = nullptr;
    e = hipMalloc(&d, bytes);
    if (e == hipSuccess) {
      rig->k[s].calib = static_cast<const float4*>(d);
      e = hipMemcpy(d, plane.data(), bytes, hipMemcpyHostToDevice);
    }
  }
  // Device-resident copy of the calibration / noise constants.
  if (e == hipSuccess) e = hipMalloc(&rig->d_k, sizeof(SensorK) * rig->n);
  if (e == hipSuccess) e = hipMemcpy(rig->d_k, rig->k, sizeof(SensorK) * rig->n, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    rig_free(rig);
    return device_error(ctx, e, "rig tables");
  }
  {
    std::lock_guard<std::mutex> g(ctx->rigs_mu);
    ctx->rigs.insert(rig);
  }
  *out = rig;
  return LPA_OK;
}

lpa_status lpa_destroy_rig(lpa_rig* rig) {
  if (!rig) return set_error(LPA_ERR_INVALID_ARG, "rig is NULL");
  lpa_ctx* ctx = rig->ctx;
  {
    std::lock_guard<std::mutex> g(ctx->rigs_mu);
    if (!ctx->rigs.erase(rig)) return set_error(LPA_ERR_INVALID_ARG, "rig is not live in its context");
  }
  // frames of this rig may still be queued or running: wait for the context's work
  if (ctx->sched) (void)lpa_drain(ctx);
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  rig_free(rig);
  (void)hipGetLastError();
  return LPA_OK;
}

lpa_status lpa_reconstruct(lpa_rig* rig, const lpa_frame* frame, const lpa_params* params,
                           const lpa_output* out, void* hip_stream) {
  try {
    return reconstruct_impl(rig, frame, params, out, hip_stream, false);
  } catch (...) {
    return set_error(LPA_ERR_INTERNAL, "unexpected exception");
  }
}

lpa_status lpa_reconstruct_plain(lpa_rig* rig, const lpa_frame* frame, const lpa_params* params,
                                 const lpa_output* out, void* hip_stream) {
  try {
    return reconstruct_impl(rig, frame, params, out, hip_stream, true);
  } catch (...) {
    return set_error(LPA_ERR_INTERNAL, "unexpected exception");
  }
}

}  // extern "C"
