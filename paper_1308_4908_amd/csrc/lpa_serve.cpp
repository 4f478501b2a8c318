// lpa_serve.cpp -- the serving loop behind lpa_submit / lpa_poll / lpa_drain:
// the scheduler policy of lpa_sched.hpp (one thread per context) driving
// the device through HipExec:
//   admission  host-resident raw planes of an admitted frame are copied into
//              a device slot on the copy stream (pinned host memory makes the
//              copy asynchronous);
//   batching   a launch is one persistent-kernel graph replay over all its
//              frames (lpa_batch.cpp), on one of two compute streams, after
//              the copies it needs (stream waits, no host blocking), so a new
//              batch overlaps the tail of the one before;
//   completion an event per batch; when it completes, its frames' counts come
//              back and their slots return to the pool.
// Calibration and noise constants stay resident in the rigs; each frame's
// result depends only on (frame, rig, params): it is bit-identical to the
// same frame reconstructed alone.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>

#include "lpa_host.hpp"
#include "lpa_sched.hpp"

namespace lpa {

// What one frame needs on the device.
struct HipJob {
  lpa_rig* rig = nullptr;
  lpa_frame frame{};
  lpa_params params{};
  lpa_output out{};
  size_t raw_bytes = 0;       // device slot for host raw planes
  void* slot = nullptr;       // device copy of host raw planes
  hipEvent_t copied = nullptr;
};

// One launch's device state.
struct HipBatch {
  hipEvent_t done = nullptr;
  int stream = 0;
};

// Device slots for host-resident frames.  A slot belongs to one frame from
// admission until its batch has completed, so a copy from pageable host
// memory (which the runtime may perform outside stream order) can never
// touch memory another frame still uses.  Slots are kept by size for reuse.
struct SlotPool {
  std::multimap<size_t, void*> free_slots;
  std::vector<void*> all;
  void* get(size_t bytes) {
    auto it = free_slots.lower_bound(bytes);
    if (it != free_slots.end() && it->first <= 2 * bytes) {
      void* p = it->second;
      free_slots.erase(it);
      return p;
    }
    void* p = nullptr;
    const size_t cap = (bytes + (1u << 20) - 1) & ~size_t((1u << 20) - 1);
    if (hipMalloc(&p, cap) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    all.push_back(p);
    sizes[p] = cap;
    return p;
  }
  void put(void* p) { free_slots.emplace(sizes[p], p); }
  void release() {
    for (void* p : all) (void)hipFree(p);
    all.clear();
    free_slots.clear();
    sizes.clear();
  }
  std::unordered_map<void*, size_t> sizes;
};

// The device side of the serving loop (the SchedCore executor).  Every
// method but thread_start runs on the scheduler thread with its lock held.
struct HipExec {
  using Job = HipJob;
  using Batch = HipBatch;

  lpa_ctx* ctx = nullptr;
  SlotPool pool;
  hipStream_t copy_stream = nullptr;
  hipStream_t compute[2] = {nullptr, nullptr};
  // per compute stream (at most one batch in flight on each): the batch's
  // output counts on the device and their pinned host copy
  uint64_t* d_stats[2] = {nullptr, nullptr};
  uint64_t* h_stats[2] = {nullptr, nullptr};
  // failure injection for tests (LPA_TEST_FAIL_AFTER=N at context creation):
  // the N-th batch launch fails from the host, before anything is enqueued,
  // as a device error would (the context fails, pending frames end with it)
  int64_t fail_after = 0;
  int64_t launches = 0;

  void thread_start() { (void)hipSetDevice(ctx->device); }
  bool failed() { return ctx->failed.load(); }
  void failure_message(char* buf, size_t n) {
    std::lock_guard<std::mutex> g(ctx->fail_mu);
    std::snprintf(buf, n, "%s", ctx->fail_msg);
  }
  void report(int32_t status, const char* msg) { (void)set_error((lpa_status)status, "%s", msg); }

  // Bytes a frame occupies on the device while in flight: host raw planes'
  // slot, pre-pass planes, its per-tile counts (8 bytes per tile of any
  // 256-pixel tile shape) and its refit marks (3 bytes per output pixel).
  size_t footprint(const Job& j) const {
    size_t b = j.raw_bytes;
    const size_t W = (size_t)j.params.out_w, H = (size_t)j.params.out_h;
    b += (W * H / 256 + W / 4 + H / 4 + 2) * 8 + W * H * 3;
    if (j.params.storage != LPA_STORE_FUSED)
      for (int s = 0; s < j.rig->n; ++s)
        b += (size_t)j.rig->desc[s].width * j.rig->desc[s].height * (j.params.storage == LPA_STORE_FP16 ? 2 : 8) +
             4096;
    return b;
  }

  // batches need one storage form and raw dtype
  uint64_t batch_key(const Job& j) const { return ((uint64_t)(uint32_t)j.params.storage << 32) | (uint32_t)j.frame.dtype; }

  // Host-resident raw planes are copied into a device slot on the copy stream.
  int32_t admit(Job& j) {
    if (j.frame.memory != LPA_MEM_HOST) return LPA_OK;
    j.slot = pool.get(j.raw_bytes);
    hipError_t e = j.slot ? hipSuccess : hipErrorOutOfMemory;
    if (e == hipSuccess) e = hipEventCreateWithFlags(&j.copied, hipEventDisableTiming);
    size_t off = 0;
    for (int s = 0; e == hipSuccess && s < j.rig->n; ++s) {
      const lpa_sensor_desc& S = j.rig->desc[s];
      const size_t es = j.frame.dtype == LPA_DTYPE_U16 ? 2 : 4;
      const size_t row = es * S.width;
      char* dst = static_cast<char*>(j.slot) + off;
      e = hipMemcpy2DAsync(dst, row, j.frame.raw[s], (size_t)j.frame.row_pitch_bytes[s], row, S.height,
                           hipMemcpyHostToDevice, copy_stream);
      j.frame.raw[s] = dst;
      j.frame.row_pitch_bytes[s] = (int64_t)row;
      off += (row * S.height + 255) / 256 * 256;
    }
    if (e == hipSuccess) e = hipEventRecord(j.copied, copy_stream);
    j.frame.memory = LPA_MEM_DEVICE;
    return e == hipSuccess ? LPA_OK : (int32_t)device_error(ctx, e, "admission copy");
  }

  // One persistent-kernel graph replay over the frames (lpa_batch.cpp), after
  // the copies they need (stream waits, no host blocking).
  int32_t launch(Job* const* jobs, int n, int stream, Batch& b) {
    b.stream = stream;
    hipStream_t st = compute[stream];
    std::vector<lpa_rig*> rigs;
    std::vector<lpa_frame> frames;
    std::vector<lpa_params> params;
    std::vector<lpa_output> outs;
    for (int i = 0; i < n; ++i) {
      Job& j = *jobs[i];
      if (j.copied) (void)hipStreamWaitEvent(st, j.copied, 0);
      rigs.push_back(j.rig);
      frames.push_back(j.frame);
      params.push_back(j.params);
      outs.push_back(j.out);
      outs.back().stats = d_stats[stream] + 2 * i;
    }
    std::vector<LaunchK> ks;
    std::vector<PlaneAlloc> planes;
    int sk = 0;
    lpa_status s = LPA_OK;
    if (fail_after > 0 && ++launches >= fail_after)
      s = device_error(ctx, hipErrorUnknown, "failure injected by LPA_TEST_FAIL_AFTER");
    // the frame footprints were charged at admission: plane scratch is not charged again
    if (s == LPA_OK)
      s = prepare_frames(ctx, n, rigs.data(), frames.data(), params.data(), outs.data(), st, &ks, &sk, &planes,
                         false);
    if (s == LPA_OK) s = launch_batch(ctx, ks, sk, st, false);
    for (const PlaneAlloc& p : planes) free_async(ctx, p.p, p.bytes, st, false);
    hipError_t e = hipSuccess;
    if (s == LPA_OK) {
      // counts to the host for lpa_result, and to callers who asked for them
      e = hipMemcpyAsync(h_stats[stream], d_stats[stream], sizeof(uint64_t) * 2 * n, hipMemcpyDeviceToHost, st);
      for (int i = 0; e == hipSuccess && i < n; ++i)
        if (jobs[i]->out.stats)
          e = hipMemcpyAsync(jobs[i]->out.stats, d_stats[stream] + 2 * i, sizeof(uint64_t) * 2,
                             hipMemcpyDeviceToDevice, st);
      if (e != hipSuccess) s = device_error(ctx, e, "count copy");
    }
    if (s == LPA_OK) {
      e = hipEventCreateWithFlags(&b.done, hipEventDisableTiming);
      if (e == hipSuccess) e = hipEventRecord(b.done, st);
      if (e != hipSuccess) s = device_error(ctx, e, "batch event");
    }
    return s;
  }

  int32_t query(Batch& b) {
    const hipError_t q = hipEventQuery(b.done);
    if (q == hipErrorNotReady) return LPA_NOT_READY;
    return q == hipSuccess ? LPA_OK : (int32_t)device_error(ctx, q, "batch execution");
  }

  void counts(const Batch& b, int i, uint64_t* n_fp64, uint64_t* n_invalid) const {
    *n_fp64 = h_stats[b.stream][2 * i];
    *n_invalid = h_stats[b.stream][2 * i + 1];
  }

  void release(Job& j) {
    if (j.copied) (void)hipEventDestroy(j.copied);
    j.copied = nullptr;
    if (j.slot) pool.put(j.slot);  // the batch that read it has completed
    j.slot = nullptr;
  }

  void release(Batch& b) {
    if (b.done) (void)hipEventDestroy(b.done);
    b.done = nullptr;
  }
};

struct Scheduler {
  HipExec exec;
  std::unique_ptr<SchedCore<HipExec>> core;
};

// Frees what serve_init made (streams, count buffers, slots) and the scheduler.
static void serve_release(Scheduler* s) {
  HipExec& x = s->exec;
  x.pool.release();
  if (x.copy_stream) (void)hipStreamDestroy(x.copy_stream);
  for (hipStream_t st : x.compute)
    if (st) (void)hipStreamDestroy(st);
  for (int i = 0; i < 2; ++i) {
    if (x.d_stats[i]) (void)hipFree(x.d_stats[i]);
    if (x.h_stats[i]) (void)hipHostFree(x.h_stats[i]);
  }
  delete s;
}

lpa_status serve_init(lpa_ctx* ctx) {
  Scheduler* s = new (std::nothrow) Scheduler();
  if (!s) return set_error(LPA_ERR_OOM, "host allocation failed");
  HipExec& x = s->exec;
  x.ctx = ctx;
  if (const char* fa = std::getenv("LPA_TEST_FAIL_AFTER")) x.fail_after = std::strtoll(fa, nullptr, 10);
  hipError_t e = hipStreamCreateWithFlags(&x.copy_stream, hipStreamNonBlocking);
  for (int i = 0; e == hipSuccess && i < 2; ++i) e = hipStreamCreateWithFlags(&x.compute[i], hipStreamNonBlocking);
  const size_t sb = sizeof(uint64_t) * 2 * SchedCore<HipExec>::kMaxBatch;
  for (int i = 0; e == hipSuccess && i < 2; ++i) {
    e = hipMalloc(&x.d_stats[i], sb);
    if (e == hipSuccess) e = hipHostMalloc(&x.h_stats[i], sb, hipHostMallocDefault);
  }
  if (e != hipSuccess) {
    serve_release(s);
    return set_error(LPA_ERR_DEVICE, "scheduler set-up: %s", hipGetErrorString(e));
  }
  s->core.reset(new (std::nothrow) SchedCore<HipExec>(x, ctx->used, ctx->budget));
  if (!s->core) {
    serve_release(s);
    return set_error(LPA_ERR_OOM, "host allocation failed");
  }
  ctx->sched = s;
  s->core->start();
  return LPA_OK;
}

void serve_shutdown(lpa_ctx* ctx) {
  Scheduler* s = ctx->sched;
  if (!s) return;
  s->core->stop();
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  s->core.reset();
  serve_release(s);
  ctx->sched = nullptr;
}

}  // namespace lpa

using namespace lpa;

extern "C" {

lpa_status lpa_submit(lpa_rig* rig, const lpa_frame* frame, const lpa_params* params, const lpa_output* out,
                      int64_t arrival_ns, uint64_t* ticket) {
  try {
    if (!rig || !ticket) return set_error(LPA_ERR_INVALID_ARG, "rig or ticket is NULL");
    lpa_ctx* ctx = rig->ctx;
    lpa_status st = check_ctx(ctx);
    if (st != LPA_OK) return st;
    Resolved R;
    if ((st = resolve_params(params, &R)) != LPA_OK) return st;
    if (R.p.mode != LPA_MODE_LPA)
      return set_error(LPA_ERR_UNSUPPORTED, "CALPA frames are reconstructed per frame (lpa_reconstruct)");
    if (R.p.flags & LPA_FLAG_PRECOMPUTED_WEIGHTS)
      return set_error(LPA_ERR_UNSUPPORTED, "pre-computed weights are a per-frame form (lpa_reconstruct)");
    if ((st = validate_frame(rig, frame, false)) != LPA_OK) return st;
    if ((st = validate_output(params, out)) != LPA_OK) return st;
    if ((st = check_batchable(rig, R, frame, out)) != LPA_OK) return st;
    HipJob j;
    j.rig = rig;
    j.frame = *frame;
    j.params = *params;
    j.out = *out;
    if (frame->memory == LPA_MEM_HOST) {
      const size_t es = frame->dtype == LPA_DTYPE_U16 ? 2 : 4;
      for (int i = 0; i < rig->n; ++i)
        j.raw_bytes += (es * rig->desc[i].width * rig->desc[i].height + 255) / 256 * 256;
    }
    const int32_t s = ctx->sched->core->submit(std::move(j), arrival_ns, ticket);
    if (s == LPA_AGAIN) return set_error(LPA_AGAIN, "admission queue full");
    if (s != LPA_OK) return set_error((lpa_status)s, "host allocation failed");
    return LPA_OK;
  } catch (...) {
    return set_error(LPA_ERR_INTERNAL, "unexpected exception");
  }
}

lpa_status lpa_poll(lpa_ctx* ctx, uint64_t ticket, lpa_result* out) {
  if (!ctx || !out) return set_error(LPA_ERR_INVALID_ARG, "context or result is NULL");
  const int32_t s = ctx->sched->core->poll(ticket, out);
  if (s == LPA_ERR_INVALID_ARG)
    return set_error(LPA_ERR_INVALID_ARG, "unknown ticket %llu", (unsigned long long)ticket);
  return (lpa_status)s;
}

lpa_status lpa_drain(lpa_ctx* ctx) {
  if (!ctx) return set_error(LPA_ERR_INVALID_ARG, "context is NULL");
  ctx->sched->core->drain();
  return ctx->failed.load() ? set_error(LPA_ERR_DEVICE, "context failed") : LPA_OK;
}

}  // extern "C"
