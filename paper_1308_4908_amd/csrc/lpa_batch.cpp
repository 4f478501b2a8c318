// lpa_batch.cpp -- batched reconstruction (one persistent launch over many
// frames, recorded into a HIP graph and replayed), the tile autotuner, and the
// context runtime set-up.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "lpa_host.hpp"

namespace lpa {

TuneKey Tuner::key_of(const lpa_rig* rig, const Resolved& R, int src_kind) {
  TuneKey k;
  k.order = R.p.order;
  k.n_scales = R.p.n_scales;
  k.n_sensors = rig->n;
  k.src_kind = src_kind;
  k.radius_q = (int)std::lround(R.p.radii[R.p.n_scales - 1] * 8.0);
  const double* O = R.p.out_affine;
  const double* A = rig->desc[0].affine;
  const double zo = std::sqrt(std::fabs(O[0] * O[4] - O[1] * O[3]));
  const double za = std::sqrt(std::fabs(A[0] * A[4] - A[1] * A[3]));
  k.zoom_q = (int)std::lround(16.0 * zo / za);
  return k;
}

// 256-lane tile shapes a batched frame may take (a batch needs one lane count).
static const int kBatchTiles[][2] = {{16, 16}, {32, 8}, {8, 32}, {64, 4}};

static int src_kind_of(const lpa_params& p, const lpa_frame& f) {
  if (p.storage == LPA_STORE_FUSED) return f.dtype == LPA_DTYPE_U16 ? SRC_RAW_U16 : SRC_RAW_F32;
  return p.storage == LPA_STORE_FP16 ? SRC_PLANE_F16 : SRC_PLANE_F32;
}

lpa_status check_batchable(const lpa_rig* rig, const Resolved& R, const lpa_frame* frame, const lpa_output* out) {
  const void* srcs[LPA_MAX_SENSORS] = {nullptr};
  int64_t pitches[LPA_MAX_SENSORS] = {0};
  LaunchK K;
  lpa_status st = LPA_ERR_UNSUPPORTED;
  for (const auto& t : kBatchTiles) {
    st = build_launch(rig, R, frame, out, src_kind_of(R.p, *frame), srcs, pitches, t[0], t[1], &K);
    if (st != LPA_ERR_UNSUPPORTED) break;
  }
  return st;
}

lpa_status prepare_frames(lpa_ctx* ctx, int n, lpa_rig* const* rigs, const lpa_frame* frames,
                          const lpa_params* params, const lpa_output* outs, hipStream_t stream,
                          std::vector<LaunchK>* ks, int* src_kind, std::vector<PlaneAlloc>* planes,
                          bool charge) {
  ks->assign(n, LaunchK());
  int sk = -1;
  std::vector<Resolved> Rs(n);
  for (int i = 0; i < n; ++i) {
    if (!rigs[i] || rigs[i]->ctx != ctx) return set_error(LPA_ERR_INVALID_ARG, "frame %d: rig missing or from another context", i);
    lpa_status st = resolve_params(&params[i], &Rs[i]);
    if (st == LPA_OK && Rs[i].p.mode != LPA_MODE_LPA)
      st = set_error(LPA_ERR_UNSUPPORTED, "frame %d: CALPA frames are reconstructed per frame", i);
    if (st == LPA_OK && (Rs[i].p.flags & LPA_FLAG_PRECOMPUTED_WEIGHTS))
      st = set_error(LPA_ERR_UNSUPPORTED, "frame %d: pre-computed weights are a per-frame form", i);
    if (st == LPA_OK) st = validate_frame(rigs[i], &frames[i], true);
    if (st == LPA_OK) st = validate_output(&params[i], &outs[i]);
    if (st != LPA_OK) return set_error(st, "frame %d: %s", i, g_last_error);
    const int k = src_kind_of(params[i], frames[i]);
    if (sk >= 0 && k != sk) return set_error(LPA_ERR_INVALID_ARG, "frames of one batch must share storage and dtype");
    sk = k;
  }
  // descriptors (and their validation) before anything is enqueued
  for (int i = 0; i < n; ++i) {
    const void* srcs[LPA_MAX_SENSORS];
    int64_t pitches[LPA_MAX_SENSORS];
    for (int s = 0; s < rigs[i]->n; ++s) {
      srcs[s] = frames[i].raw[s];
      pitches[s] = frames[i].row_pitch_bytes[s];
    }
    const TuneChoice tc = ctx->tuner.choose(Tuner::key_of(rigs[i], Rs[i], sk));
    int tw = tc.tile_w, th = tc.tile_h;
    lpa_status st = build_launch(rigs[i], Rs[i], &frames[i], &outs[i], sk, srcs, pitches, tw, th, &(*ks)[i]);
    if (st == LPA_ERR_UNSUPPORTED && tw * th == 256)
      for (const auto& t : kBatchTiles) {
        st = build_launch(rigs[i], Rs[i], &frames[i], &outs[i], sk, srcs, pitches, t[0], t[1], &(*ks)[i]);
        if (st != LPA_ERR_UNSUPPORTED) break;
      }
    if (st != LPA_OK) return set_error(st, "frame %d: %s", i, g_last_error);
  }
  *src_kind = sk;
  if (sk == SRC_PLANE_F32 || sk == SRC_PLANE_F16) {
    // the planes only, carved from one allocation (one stream-ordered
    // allocation per batch, not one per sensor): the batch graph's pre-pass
    // node fills them
    const int64_t es = sk == SRC_PLANE_F16 ? 2 : 8;
    size_t bytes = 0;
    for (int i = 0; i < n; ++i)
      for (int s = 0; s < rigs[i]->n; ++s)
        bytes += (size_t)((rigs[i]->k[s].width * es + 255) / 256 * 256) * rigs[i]->k[s].height;
    void* buf = nullptr;
    lpa_status st = alloc_async(ctx, bytes, stream, &buf, charge);
    if (st != LPA_OK) return st;
    planes->push_back({buf, bytes});
    size_t at = 0;
    for (int i = 0; i < n; ++i)
      for (int s = 0; s < rigs[i]->n; ++s) {
        const int64_t pitch = (rigs[i]->k[s].width * es + 255) / 256 * 256;
        (*ks)[i].s[s].src = static_cast<char*>(buf) + at;
        (*ks)[i].s[s].pitch = pitch;
        at += (size_t)pitch * rigs[i]->k[s].height;
      }
  }
  return LPA_OK;
}

lpa_status launch_table(lpa_ctx* ctx, const std::vector<LaunchK>& ks, int src_kind, int block, int lds,
                        int refit_lds, int grid, int64_t total, hipStream_t stream);

static void slot_release(BatchSlot& sl) {
  if (sl.exec) (void)hipGraphExecDestroy(sl.exec);
  if (sl.graph) (void)hipGraphDestroy(sl.graph);
  sl.graph = nullptr;
  if (sl.h_buf) (void)hipHostFree(sl.h_buf);
  if (sl.d_buf) (void)hipFree(sl.d_buf);
  sl.exec = nullptr;
  sl.h_buf = nullptr;
  sl.d_buf = nullptr;
  sl.cap = 0;
}

lpa_status launch_batch(lpa_ctx* ctx, const std::vector<LaunchK>& ks_in, int src_kind, hipStream_t stream,
                        bool charge) {
  std::vector<LaunchK> ks = ks_in;
  int block = ks[0].tile_w * ks[0].tile_h;
  int lds = 0, refit_lds = 0;
  int64_t total = 0;
  for (const LaunchK& K : ks) {
    if (K.tile_w * K.tile_h != block) return set_error(LPA_ERR_INTERNAL, "batch tiles differ in lane count");
    for (int s = 0; s < K.n_sensors; ++s)
      if (!K.s[s].raw) return set_error(LPA_ERR_INTERNAL, "batch frame without raw planes");
    lds = std::max(lds, K.lds_floats2);
    refit_lds = std::max(refit_lds, K.refit_lds * (K.s[0].raw_f32 ? 4 : 2));
    total += (int64_t)K.tiles_x * K.tiles_y;
  }
  if (total > (int64_t)INT32_MAX) return set_error(LPA_ERR_UNSUPPORTED, "batch exceeds 2^31 tiles");
  const int grid = (int)std::min<int64_t>(total, (int64_t)ctx->n_cu * 4);
  // per-tile counts for the frames whose outputs ask for them, and the refit
  // marks (3 bytes per output pixel) of the frames with an accuracy target
  void* cbuf = nullptr;
  void* rbuf = nullptr;
  size_t cbytes = 0, rbytes = 0;
  bool counts = false;
  for (const LaunchK& K : ks) {
    counts = counts || K.frame_stats;
    if (std::isfinite(K.risk_max)) rbytes += (size_t)K.out_w * K.out_h * 3;
  }
  if (counts) {
    cbytes = (size_t)total * 2 * sizeof(uint32_t);
    lpa_status cs = alloc_async(ctx, cbytes, stream, &cbuf, charge);
    if (cs != LPA_OK) return cs;
    int64_t at = 0;
    for (LaunchK& K : ks) {
      if (K.frame_stats) K.tile_stats = static_cast<uint32_t*>(cbuf) + 2 * at;
      at += (int64_t)K.tiles_x * K.tiles_y;
    }
  }
  if (rbytes) {
    lpa_status rs = alloc_async(ctx, rbytes, stream, &rbuf, charge);
    if (rs != LPA_OK) {
      free_async(ctx, cbuf, cbytes, stream, charge);
      return rs;
    }
    size_t at = 0;
    for (LaunchK& K : ks) {
      if (!std::isfinite(K.risk_max)) continue;
      K.refit_map = static_cast<uint8_t*>(rbuf) + at;
      K.refit_pitch = (int64_t)3 * K.out_w;
      at += (size_t)K.out_w * K.out_h * 3;
    }
  }
  lpa_status st = launch_table(ctx, ks, src_kind, block, lds, refit_lds, grid, total, stream);
  free_async(ctx, rbuf, rbytes, stream, charge);
  free_async(ctx, cbuf, cbytes, stream, charge);
  return st;
}

// Copy the table into a slot and replay (or build) its graph: the table copy,
// the queue reset, the persistent kernel, the FP64 refit and the count
// reduction.
lpa_status launch_table(lpa_ctx* ctx, const std::vector<LaunchK>& ks, int src_kind, int block, int lds,
                        int refit_lds, int grid, int64_t total, hipStream_t stream) {
  const int n = (int)ks.size();

  std::lock_guard<std::mutex> g(ctx->batch_mu);
  BatchSlot& sl = ctx->slots[ctx->next_slot];
  ctx->next_slot = (ctx->next_slot + 1) % (int)ctx->slots.size();
  hipError_t e;
  if (sl.used && (e = hipEventSynchronize(sl.done)) != hipSuccess) return device_error(ctx, e, "batch slot wait");
  if (sl.cap < n) {
    slot_release(sl);
    int cap = 64;
    while (cap < n) cap *= 2;
    BatchLayout L(cap);
    if ((e = hipHostMalloc(&sl.h_buf, L.copy_bytes, hipHostMallocDefault)) != hipSuccess ||
        (e = hipMalloc(&sl.d_buf, L.total_bytes)) != hipSuccess) {
      slot_release(sl);
      return set_error(LPA_ERR_OOM, "batch table allocation: %s", hipGetErrorString(e));
    }
    sl.cap = cap;
  }
  BatchLayout L(sl.cap);
  char* h = static_cast<char*>(sl.h_buf);
  BatchHeader hdr;
  hdr.n_frames = n;
  hdr.pad_ = 0;
  hdr.total_tiles = total;
  std::memcpy(h, &hdr, sizeof(hdr));
  std::memcpy(h + L.frames_off, ks.data(), sizeof(LaunchK) * n);
  int64_t* first = reinterpret_cast<int64_t*>(h + L.first_off);
  int64_t acc = 0;
  for (int i = 0; i < n; ++i) {
    first[i] = acc;
    acc += (int64_t)ks[i].tiles_x * ks[i].tiles_y;
  }
  // The graph depends on the source kind, block, grid and capacity; a batch
  // whose frames need another LDS size updates the two kernel nodes of the
  // instantiated graph.
  const int raw_f32 = ks[0].s[0].raw_f32;  // one dtype per batch
  const int64_t sig[5] = {src_kind, block, grid, sl.cap, raw_f32};
  char* d = static_cast<char*>(sl.d_buf);
  const auto* d_hdr = reinterpret_cast<const BatchHeader*>(d);
  const auto* d_frames = reinterpret_cast<const LaunchK*>(d + L.frames_off);
  const auto* d_first = reinterpret_cast<const int64_t*>(d + L.first_off);
  auto* d_queue = reinterpret_cast<int32_t*>(d + L.queue_off);
  // the refit takes one workgroup per output block of the frames that have
  // refits, each of the 8 XCDs an eighth of every frame's blocks: the grid is
  // 8 x the largest per-XCD count (refit_batch_kernel)
  int64_t per_xcd[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (const LaunchK& K : ks)
    if (K.refit_map) {
      const int64_t nb = (int64_t)((K.out_w + K.refit_bw - 1) / K.refit_bw) * ((K.out_h + K.refit_bh - 1) / K.refit_bh);
      for (int x = 0; x < 8; ++x) per_xcd[x] += nb * (x + 1) / 8 - nb * x / 8;
    }
  const int64_t refit_blocks = 8 * std::max<int64_t>(*std::max_element(per_xcd, per_xcd + 8), 1);
  if (refit_blocks > (int64_t)INT32_MAX) return set_error(LPA_ERR_UNSUPPORTED, "batch exceeds 2^31 refit blocks");
  const int refit_grid = (int)refit_blocks;
  bool rebuild = !sl.exec || std::memcmp(sig, sl.sig, sizeof(sig)) != 0;
  if (!rebuild && (sl.lds != lds || sl.refit_lds != refit_lds || sl.refit_grid != refit_grid)) {
    // another LDS size or refit grid: update the two nodes in place; a
    // runtime that refuses the update gets a new graph instead
    if (lpa_k_batch_graph_set_lds(sl.exec, sl.fit_node, sl.refit_node, d_hdr, d_frames, d_first, d_queue, src_kind,
                                  block, lds, refit_lds, grid, refit_grid, raw_f32) == 0) {
      sl.lds = lds;
      sl.refit_lds = refit_lds;
      sl.refit_grid = refit_grid;
    }
    else {
      (void)hipGetLastError();
      rebuild = true;
    }
  }
  if (rebuild) {
    if (sl.exec) (void)hipGraphExecDestroy(sl.exec);
    if (sl.graph) (void)hipGraphDestroy(sl.graph);
    sl.exec = nullptr;
    sl.graph = nullptr;
    if (lpa_k_batch_graph(&sl.graph, &sl.fit_node, &sl.refit_node, d, h, L.copy_bytes, d_hdr, d_frames, d_first,
                          d_queue, src_kind, block, lds, refit_lds, grid, refit_grid, sl.cap, raw_f32) != 0)
      return device_error(ctx, hipGetLastError(), "batch graph");
    e = hipGraphInstantiate(&sl.exec, sl.graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      sl.exec = nullptr;
      return device_error(ctx, e, "graph instantiate");
    }
    std::memcpy(sl.sig, sig, sizeof(sig));
    sl.lds = lds;
    sl.refit_lds = refit_lds;
    sl.refit_grid = refit_grid;
  }
  if ((e = hipGraphLaunch(sl.exec, stream)) != hipSuccess) return device_error(ctx, e, "graph launch");
  if ((e = hipEventRecord(sl.done, stream)) != hipSuccess) return device_error(ctx, e, "event record");
  sl.used = true;
  return LPA_OK;
}

lpa_status ctx_init_runtime(lpa_ctx* ctx) {
  hipError_t e;
  ctx->slots.resize(4);
  for (BatchSlot& sl : ctx->slots)
    if ((e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming)) != hipSuccess)
      return set_error(LPA_ERR_DEVICE, "event create: %s", hipGetErrorString(e));
  return serve_init(ctx);
}

void ctx_shutdown_runtime(lpa_ctx* ctx) {
  serve_shutdown(ctx);
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  for (BatchSlot& sl : ctx->slots) {
    slot_release(sl);
    if (sl.done) (void)hipEventDestroy(sl.done);
  }
  ctx->slots.clear();
}

}  // namespace lpa

using namespace lpa;

extern "C" lpa_status lpa_reconstruct_batch(lpa_ctx* ctx, int32_t n, lpa_rig* const* rigs,
                                            const lpa_frame* frames, const lpa_params* params,
                                            const lpa_output* outs, void* hip_stream) {
  try {
    lpa_status st = check_ctx(ctx);
    if (st != LPA_OK) return st;
    if (n < 1 || n > 4096 || !rigs || !frames || !params || !outs)
      return set_error(LPA_ERR_INVALID_ARG, "batch needs 1..4096 frames and non-NULL arrays");
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return device_error(ctx, e, "hipSetDevice");
    hipStream_t hs = static_cast<hipStream_t>(hip_stream);
    std::vector<LaunchK> ks;
    std::vector<PlaneAlloc> planes;
    int sk = 0;
    st = prepare_frames(ctx, n, rigs, frames, params, outs, hs, &ks, &sk, &planes);
    if (st == LPA_OK) st = launch_batch(ctx, ks, sk, hs);
    for (const PlaneAlloc& p : planes) free_async(ctx, p.p, p.bytes, hs);
    return st;
  } catch (...) {
    return set_error(LPA_ERR_INTERNAL, "unexpected exception");
  }
}
