// lpa_tune.cpp -- the launch-shape autotuner: measures every candidate
// (tile shape x register budget) on a caller's frame and keeps the fastest for
// the frame's class; choices persist to a small JSON file.
//
// Candidates all have 256 lanes per workgroup, so tuned frames of any class
// can share one persistent batch launch.  The per-pixel arithmetic does not
// depend on the choice: every candidate produces bit-identical output.
#include <cmath>
#include <cstdio>
#include <cstring>

#include "lpa_host.hpp"

namespace lpa {

static const int kCandTiles[][2] = {{16, 16}, {32, 8}, {8, 32}, {64, 4}};

static lpa_status time_launch(lpa_ctx* ctx, LaunchK& K, hipStream_t st, int reps, double* ms) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e != hipSuccess) return device_error(ctx, e, "tuner events");
  lpa_status s = LPA_OK;
  if (lpa_k_fit(&K, st) != 0) s = device_error(ctx, hipGetLastError(), "tuner warm-up launch");
  if (s == LPA_OK) {
    (void)hipEventRecord(e0, st);
    for (int r = 0; r < reps && s == LPA_OK; ++r)
      if (lpa_k_fit(&K, st) != 0) s = device_error(ctx, hipGetLastError(), "tuner launch");
    (void)hipEventRecord(e1, st);
    if ((e = hipEventSynchronize(e1)) != hipSuccess) s = device_error(ctx, e, "tuner sync");
    float f = 0.f;
    if (s == LPA_OK && hipEventElapsedTime(&f, e0, e1) == hipSuccess) *ms = f / reps;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return s;
}

}  // namespace lpa

using namespace lpa;

extern "C" {

lpa_status lpa_autotune(lpa_rig* rig, const lpa_frame* frame, const lpa_params* params, const lpa_output* out,
                        void* hip_stream, int32_t reps, lpa_tune_result* res) {
  try {
    if (!rig) return set_error(LPA_ERR_INVALID_ARG, "rig is NULL");
    lpa_ctx* ctx = rig->ctx;
    lpa_status st = check_ctx(ctx);
    if (st != LPA_OK) return st;
    Resolved R;
    if ((st = resolve_params(params, &R)) != LPA_OK) return st;
    if (R.p.mode != LPA_MODE_LPA)
      return set_error(LPA_ERR_UNSUPPORTED, "CALPA frames are reconstructed per frame (lpa_reconstruct)");
    if (R.p.flags & LPA_FLAG_PRECOMPUTED_WEIGHTS)
      return set_error(LPA_ERR_UNSUPPORTED, "pre-computed weights use a fixed 16x16 launch (not tuned)");
    if ((st = validate_frame(rig, frame, true)) != LPA_OK) return st;
    if ((st = validate_output(params, out)) != LPA_OK) return st;
    if (reps < 1 || reps > 1000) return set_error(LPA_ERR_INVALID_ARG, "reps %d outside 1..1000", reps);
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return device_error(ctx, e, "hipSetDevice");
    hipStream_t hs = static_cast<hipStream_t>(hip_stream);
    const void* srcs[LPA_MAX_SENSORS];
    int64_t pitches[LPA_MAX_SENSORS];
    void* planes[LPA_MAX_SENSORS] = {nullptr};
    size_t plane_bytes[LPA_MAX_SENSORS] = {0};
    int src_kind;
    if (R.p.storage == LPA_STORE_FUSED) {
      src_kind = frame->dtype == LPA_DTYPE_U16 ? SRC_RAW_U16 : SRC_RAW_F32;
      for (int s = 0; s < rig->n; ++s) {
        srcs[s] = frame->raw[s];
        pitches[s] = frame->row_pitch_bytes[s];
      }
    } else {
      src_kind = R.p.storage == LPA_STORE_FP16 ? SRC_PLANE_F16 : SRC_PLANE_F32;
      st = run_prepass(rig, frame, R.p.storage == LPA_STORE_FP16, hs, planes, plane_bytes, srcs, pitches);
    }
    TuneChoice best;
    double best_ms = INFINITY, default_ms = INFINITY;
    int tried = 0;
    for (int ti = 0; st == LPA_OK && ti < 4; ++ti) {
      for (int occ : {0, 4}) {
        if (occ == 4 && R.p.order != 2) continue;
        LaunchK K;
        lpa_status b =
            build_launch(rig, R, frame, out, src_kind, srcs, pitches, kCandTiles[ti][0], kCandTiles[ti][1], &K);
        if (b == LPA_ERR_UNSUPPORTED) continue;
        if (b != LPA_OK) {
          st = b;
          break;
        }
        K.occupancy = occ;
        K.risk_max = INFINITY;  // the fit alone is timed (the refit launch does not depend on the shape)
        double ms = INFINITY;
        if ((st = time_launch(ctx, K, hs, reps, &ms)) != LPA_OK) break;
        ++tried;
        if (ti == 0 && occ == 0) default_ms = ms;
        if (ms < best_ms) {
          best_ms = ms;
          best.tile_w = kCandTiles[ti][0];
          best.tile_h = kCandTiles[ti][1];
          best.occupancy = occ;
        }
      }
    }
    for (int s = 0; s < rig->n; ++s) free_async(ctx, planes[s], plane_bytes[s], hs);
    if (st != LPA_OK) return st;
    if (!tried) return set_error(LPA_ERR_UNSUPPORTED, "no candidate launch shape fits this frame");
    ctx->tuner.set(Tuner::key_of(rig, R, src_kind), best);
    if (res) {
      res->tile_w = best.tile_w;
      res->tile_h = best.tile_h;
      res->occupancy = best.occupancy;
      res->n_candidates = tried;
      res->ms_best = best_ms;
      res->ms_default = default_ms;
    }
    (void)hipStreamSynchronize(hs);
    return LPA_OK;
  } catch (...) {
    return set_error(LPA_ERR_INTERNAL, "unexpected exception");
  }
}

lpa_status lpa_tuner_save(lpa_ctx* ctx, const char* path) {
  if (!ctx || !path) return set_error(LPA_ERR_INVALID_ARG, "context or path is NULL");
  FILE* f = std::fopen(path, "w");
  if (!f) return set_error(LPA_ERR_INVALID_ARG, "cannot write %s", path);
  hipDeviceProp_t prop;
  const char* arch = hipGetDeviceProperties(&prop, ctx->device) == hipSuccess ? prop.gcnArchName : "unknown";
  std::fprintf(f, "{\"arch\": \"%s\", \"entries\": [\n", arch);
  const auto tab = ctx->tuner.snapshot();
  size_t i = 0;
  for (const auto& kv : tab) {
    const TuneKey& k = kv.first;
    const TuneChoice& c = kv.second;
    std::fprintf(f,
                 " {\"order\": %d, \"n_scales\": %d, \"n_sensors\": %d, \"src\": %d, \"radius_q\": %d, "
                 "\"zoom_q\": %d, \"tile_w\": %d, \"tile_h\": %d, \"occupancy\": %d}%s\n",
                 k.order, k.n_scales, k.n_sensors, k.src_kind, k.radius_q, k.zoom_q, c.tile_w, c.tile_h,
                 c.occupancy, ++i < tab.size() ? "," : "");
  }
  std::fprintf(f, "]}\n");
  std::fclose(f);
  return LPA_OK;
}

lpa_status lpa_tuner_load(lpa_ctx* ctx, const char* path) {
  if (!ctx || !path) return set_error(LPA_ERR_INVALID_ARG, "context or path is NULL");
  FILE* f = std::fopen(path, "r");
  if (!f) return set_error(LPA_ERR_INVALID_ARG, "cannot read %s", path);
  char line[512];
  int loaded = 0;
  while (std::fgets(line, sizeof(line), f)) {
    TuneKey k;
    TuneChoice c;
    if (std::sscanf(line,
                    " {\"order\": %d, \"n_scales\": %d, \"n_sensors\": %d, \"src\": %d, \"radius_q\": %d, "
                    "\"zoom_q\": %d, \"tile_w\": %d, \"tile_h\": %d, \"occupancy\": %d}",
                    &k.order, &k.n_scales, &k.n_sensors, &k.src_kind, &k.radius_q, &k.zoom_q, &c.tile_w,
                    &c.tile_h, &c.occupancy) == 9) {
      const bool ok_tile = c.tile_w > 0 && c.tile_h > 0 && c.tile_w % 2 == 0 && c.tile_h % 2 == 0 &&
                           c.tile_w * c.tile_h == 256;
      if (!ok_tile || (c.occupancy != 0 && c.occupancy != 4)) {
        std::fclose(f);
        return set_error(LPA_ERR_INVALID_ARG, "bad tuner entry in %s", path);
      }
      ctx->tuner.set(k, c);
      ++loaded;
    }
  }
  std::fclose(f);
  return LPA_OK;
}

}  // extern "C"
