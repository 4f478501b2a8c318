// lpa_noalloc.cpp -- lpa_reconstruct_noalloc: the fused single-frame
// reconstruction with its scratch in a static device array, for callers that
// cannot allocate device memory.
//
// The fused form's only scratch is the refit marks (3 bytes per output pixel,
// written by the fit launch, read by the FP64 refit launch) and, when the
// output asks for counts, the per-tile counts (8 bytes per tile).  Here both
// live in `scratch`, a file-scope device array of kNoAllocScratchBytes that
// each GPU holds until the process ends.  Host code never passes the array's
// name to a kernel: lpa_create_ctx calls noalloc_init_device with the
// context's device current, which takes the array's device address with
// hipGetSymbolAddress and keeps it per device; the launches use that address.
// Every call on one GPU shares its array: the fit rewrites every mark and
// every tile count before they are read, so nothing needs clearing, but calls
// that overlap on one GPU (different streams, threads) race.
#include <cmath>
#include <mutex>

#include "lpa_host.hpp"

namespace lpa {

constexpr size_t kNoAllocScratchBytes = size_t(16) << 20;
constexpr int kNoAllocMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
std::mutex g_mu;
void* g_scratch_ptr[kNoAllocMaxDevices] = {};
}  // namespace

lpa_status noalloc_init_device(int device) {
  if (device < 0 || device >= kNoAllocMaxDevices)
    return set_error(LPA_ERR_UNSUPPORTED, "device %d: the allocation-free entry point serves devices 0..%d", device,
                     kNoAllocMaxDevices - 1);
  std::lock_guard<std::mutex> g(g_mu);
  if (g_scratch_ptr[device]) return LPA_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    return set_error(LPA_ERR_DEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", device, hipGetErrorString(e));
  g_scratch_ptr[device] = p;
  return LPA_OK;
}

static void* scratch_of(int device) {
  if (device < 0 || device >= kNoAllocMaxDevices) return nullptr;
  std::lock_guard<std::mutex> g(g_mu);
  return g_scratch_ptr[device];
}

}  // namespace lpa

using namespace lpa;

extern "C" lpa_status lpa_reconstruct_noalloc(lpa_rig* rig, const lpa_frame* frame, const lpa_params* params,
                                              const lpa_output* out, void* hip_stream) {
  try {
    if (!rig) return set_error(LPA_ERR_INVALID_ARG, "rig is NULL");
    lpa_ctx* ctx = rig->ctx;
    lpa_status st = check_ctx(ctx);
    if (st != LPA_OK) return st;
    Resolved R;
    if ((st = resolve_params(params, &R)) != LPA_OK) return st;
    if ((st = validate_frame(rig, frame, true)) != LPA_OK) return st;
    if ((st = validate_output(params, out)) != LPA_OK) return st;
    if (R.p.mode != LPA_MODE_LPA)
      return set_error(LPA_ERR_UNSUPPORTED, "the allocation-free form reconstructs mode LPA (CALPA needs gradient and "
                                            "steering planes)");
    if (R.p.storage != LPA_STORE_FUSED)
      return set_error(LPA_ERR_UNSUPPORTED, "the allocation-free form reads raw samples (storage FUSED): the pre-pass "
                                            "forms need planes");
    if (R.p.flags & LPA_FLAG_PRECOMPUTED_WEIGHTS)
      return set_error(LPA_ERR_UNSUPPORTED, "the allocation-free form computes window weights (their tables are "
                                            "allocated on first use)");
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return device_error(ctx, e, "hipSetDevice");
    char* base = static_cast<char*>(scratch_of(ctx->device));
    if (!base) return set_error(LPA_ERR_INTERNAL, "no scratch address for device %d", ctx->device);

    const int src_kind = frame->dtype == LPA_DTYPE_U16 ? SRC_RAW_U16 : SRC_RAW_F32;
    const void* srcs[LPA_MAX_SENSORS];
    int64_t pitches[LPA_MAX_SENSORS];
    for (int s = 0; s < rig->n; ++s) {
      srcs[s] = frame->raw[s];
      pitches[s] = frame->row_pitch_bytes[s];
    }
    const TuneChoice tc = ctx->tuner.choose(Tuner::key_of(rig, R, src_kind));
    LaunchK K;
    if ((st = build_launch_fit(rig, R, frame, out, src_kind, srcs, pitches, tc.tile_w, tc.tile_h, &K)) != LPA_OK)
      return st;
    K.occupancy = tc.occupancy;
    const int64_t tiles = (int64_t)K.tiles_x * K.tiles_y;
    const size_t map_bytes = std::isfinite(K.risk_max) ? ((size_t)K.out_w * K.out_h * 3 + 255) / 256 * 256 : 0;
    const size_t stat_bytes = out->stats ? (size_t)tiles * 2 * sizeof(uint32_t) : 0;
    if (map_bytes + stat_bytes > kNoAllocScratchBytes)
      return set_error(LPA_ERR_UNSUPPORTED,
                       "output %dx%d needs %zu bytes of scratch; the allocation-free form holds %zu (about %zu "
                       "output pixels)",
                       K.out_w, K.out_h, map_bytes + stat_bytes, kNoAllocScratchBytes, kNoAllocScratchBytes / 4);
    if (map_bytes) {
      K.refit_map = reinterpret_cast<uint8_t*>(base);
      K.refit_pitch = (int64_t)3 * K.out_w;
    }
    if (stat_bytes) K.tile_stats = reinterpret_cast<uint32_t*>(base + map_bytes);
    hipStream_t hs = static_cast<hipStream_t>(hip_stream);
    if (lpa_k_fit(&K, hs) != 0) return device_error(ctx, hipGetLastError(), "fit launch");
    if (map_bytes && lpa_k_refit(&K, hs) != 0) return device_error(ctx, hipGetLastError(), "refit launch");
    if (stat_bytes && lpa_k_stats_sum(K.tile_stats, tiles, out->stats, hs) != 0)
      return device_error(ctx, hipGetLastError(), "count reduction");
    return LPA_OK;
  } catch (...) {
    return set_error(LPA_ERR_INTERNAL, "unexpected exception");
  }
}
