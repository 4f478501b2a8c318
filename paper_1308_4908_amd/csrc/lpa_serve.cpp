// lpa_serve.cpp -- the serving loop behind lpa_submit / lpa_poll / lpa_drain.
//
// One scheduler thread per context:
//   admission  frames wait in a bounded FIFO until the HBM budget admits
//              them; host-resident raw planes are then copied into a device
//              slot on the copy stream (pinned host memory makes the copy
//              asynchronous);
//   batching   every admitted frame that is not yet running joins the next
//              launch: one persistent-kernel graph replay over all of them
//              (lpa_batch.cpp), on one of two compute streams, after the
//              copies it needs (stream waits, no host blocking), so a new
//              batch overlaps the tail of the one before;
//   completion an event per batch; when it completes, its frames get their
//              timestamps and status and their slots return to the budget.
// Calibration and noise constants stay resident in the rigs; each frame's
// result depends only on (frame, rig, params): it is bit-identical to the
// same frame reconstructed alone.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>

#include "lpa_host.hpp"

namespace lpa {

static int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

struct Request {
  uint64_t ticket;
  lpa_rig* rig;
  lpa_frame frame;
  lpa_params params;
  lpa_output out;
  int64_t arrival_ns, admit_ns = 0, start_ns = 0, done_ns = 0;
  size_t raw_bytes = 0;       // device slot for host raw planes
  size_t reserved = 0;        // bytes charged to the budget at admission
  void* slot = nullptr;       // device copy of host raw planes
  hipEvent_t copied = nullptr;
  int32_t status = LPA_NOT_READY;
  int32_t batch_size = 0;
  uint64_t n_fp64 = 0, n_invalid = 0;  // the frame's output counts
};

struct Batch {
  std::vector<Request*> reqs;
  std::vector<PlaneAlloc> planes;
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

struct Scheduler {
  lpa_ctx* ctx = nullptr;
  SlotPool pool;
  std::mutex mu;
  std::condition_variable cv;       // wakes the scheduler
  std::condition_variable cv_done;  // wakes lpa_drain
  std::deque<Request*> waiting;     // submitted, not admitted
  std::deque<Request*> admitted;    // admitted, not launched
  std::vector<Batch> inflight;
  std::unordered_map<uint64_t, lpa_result> results;
  uint64_t next_ticket = 1;
  size_t pending = 0;               // submitted and not finished
  bool stop = false;
  hipStream_t copy_stream = nullptr;
  hipStream_t compute[2] = {nullptr, nullptr};
  // per compute stream (at most one batch in flight on each): the batch's
  // output counts on the device and their pinned host copy
  uint64_t* d_stats[2] = {nullptr, nullptr};
  uint64_t* h_stats[2] = {nullptr, nullptr};
  std::thread worker;
  // failure injection for tests (LPA_TEST_FAIL_AFTER=N at context creation):
  // the N-th batch launch fails from the host, before anything is enqueued,
  // as a device error would (the context fails, pending frames end with it)
  int64_t fail_after = 0;
  int64_t launches = 0;
  static constexpr size_t kQueueCap = 1024;
  static constexpr int kMaxInflight = 2;
  static constexpr int kMaxBatch = 64;

  void finish(Request* r, int32_t status) {
    r->status = status;
    r->done_ns = now_ns();
    lpa_result res;
    res.status = status;
    res.batch_size = r->batch_size;
    res.t_arrival_ns = r->arrival_ns;
    res.t_admit_ns = r->admit_ns;
    res.t_start_ns = r->start_ns;
    res.t_done_ns = r->done_ns;
    res.n_fp64 = r->n_fp64;
    res.n_invalid = r->n_invalid;
    results[r->ticket] = res;
    if (r->copied) (void)hipEventDestroy(r->copied);
    if (r->slot) pool.put(r->slot);  // the batch that read it has completed
    ctx->used.fetch_sub(r->reserved);
    delete r;
    --pending;
    // every terminal path (completion, rejection at admission, launch failure)
    // must wake lpa_drain, which waits for pending == 0
    cv_done.notify_all();
  }

  // Bytes a frame occupies on the device while in flight: host raw planes'
  // slot, pre-pass planes, its per-tile counts (8 bytes per tile of any
  // 256-pixel tile shape) and its refit marks (3 bytes per output pixel).
  size_t footprint(const Request* r) const {
    size_t b = r->raw_bytes;
    const size_t W = (size_t)r->params.out_w, H = (size_t)r->params.out_h;
    b += (W * H / 256 + W / 4 + H / 4 + 2) * 8 + W * H * 3;  // + the refit marks
    if (r->params.storage != LPA_STORE_FUSED)
      for (int s = 0; s < r->rig->n; ++s)
        b += (size_t)r->rig->desc[s].width * r->rig->desc[s].height * (r->params.storage == LPA_STORE_FP16 ? 2 : 8) + 4096;
    return b;
  }

  // Admit waiting frames in order while the budget allows (caller holds mu).
  void admit() {
    while (!waiting.empty()) {
      Request* r = waiting.front();
      const size_t need = footprint(r);
      // Served frames in flight will return their memory; without any, what
      // the context holds (rig-resident calibration planes and weight tables)
      // stays, and a frame that does not fit beside it never will.
      if (ctx->used.load() + need > ctx->budget) {
        if (!admitted.empty() || !inflight.empty()) return;
        waiting.pop_front();
        set_error(LPA_ERR_OOM, "frame needs %zu bytes; %zu of the budget of %zu are held", need,
                  ctx->used.load(), ctx->budget);
        finish(r, LPA_ERR_OOM);
        continue;
      }
      ctx->used.fetch_add(need);
      r->reserved = need;
      waiting.pop_front();
      r->admit_ns = now_ns();
      if (r->frame.memory == LPA_MEM_HOST) {
        r->slot = pool.get(r->raw_bytes);
        hipError_t e = r->slot ? hipSuccess : hipErrorOutOfMemory;
        if (e == hipSuccess) e = hipEventCreateWithFlags(&r->copied, hipEventDisableTiming);
        size_t off = 0;
        for (int s = 0; e == hipSuccess && s < r->rig->n; ++s) {
          const lpa_sensor_desc& S = r->rig->desc[s];
          const size_t es = r->frame.dtype == LPA_DTYPE_U16 ? 2 : 4;
          const size_t row = es * S.width;
          char* dst = static_cast<char*>(r->slot) + off;
          e = hipMemcpy2DAsync(dst, row, r->frame.raw[s], (size_t)r->frame.row_pitch_bytes[s], row, S.height,
                               hipMemcpyHostToDevice, copy_stream);
          r->frame.raw[s] = dst;
          r->frame.row_pitch_bytes[s] = (int64_t)row;
          off += (row * S.height + 255) / 256 * 256;
        }
        if (e == hipSuccess) e = hipEventRecord(r->copied, copy_stream);
        r->frame.memory = LPA_MEM_DEVICE;
        if (e != hipSuccess) {
          device_error(ctx, e, "admission copy");
          finish(r, LPA_ERR_DEVICE);
          continue;
        }
      }
      admitted.push_back(r);
    }
  }

  // Launch the admitted frames as one batch (caller holds mu).
  void launch() {
    const int n = (int)std::min<size_t>(admitted.size(), kMaxBatch);
    // batches need one storage form and dtype: take the longest prefix that shares them
    int take = 1;
    while (take < n && admitted[take]->params.storage == admitted[0]->params.storage &&
           admitted[take]->frame.dtype == admitted[0]->frame.dtype)
      ++take;
    Batch b;
    b.reqs.assign(admitted.begin(), admitted.begin() + take);
    admitted.erase(admitted.begin(), admitted.begin() + take);
    // the compute stream no batch in flight uses (launch runs only with
    // fewer than kMaxInflight = 2 batches in flight)
    b.stream = (!inflight.empty() && inflight.front().stream == 0) ? 1 : 0;
    hipStream_t st = compute[b.stream];
    std::vector<lpa_rig*> rigs;
    std::vector<lpa_frame> frames;
    std::vector<lpa_params> params;
    std::vector<lpa_output> outs;
    for (Request* r : b.reqs) {
      if (r->copied) (void)hipStreamWaitEvent(st, r->copied, 0);
      rigs.push_back(r->rig);
      frames.push_back(r->frame);
      params.push_back(r->params);
      outs.push_back(r->out);
      outs.back().stats = d_stats[b.stream] + 2 * (frames.size() - 1);
      r->batch_size = take;
    }
    std::vector<LaunchK> ks;
    int sk = 0;
    const int64_t t = now_ns();
    lpa_status s = LPA_OK;
    if (fail_after > 0 && ++launches >= fail_after)
      s = device_error(ctx, hipErrorUnknown, "failure injected by LPA_TEST_FAIL_AFTER");
    // the frame footprints were charged at admission: plane scratch is not charged again
    if (s == LPA_OK)
      s = prepare_frames(ctx, take, rigs.data(), frames.data(), params.data(), outs.data(), st, &ks, &sk, &b.planes,
                         false);
    if (s == LPA_OK) s = launch_batch(ctx, ks, sk, st, false);
    for (const PlaneAlloc& p : b.planes) free_async(ctx, p.p, p.bytes, st, false);
    b.planes.clear();
    hipError_t e = hipSuccess;
    if (s == LPA_OK) {
      // counts to the host for lpa_result, and to callers who asked for them
      e = hipMemcpyAsync(h_stats[b.stream], d_stats[b.stream], sizeof(uint64_t) * 2 * take, hipMemcpyDeviceToHost, st);
      for (int i = 0; e == hipSuccess && i < take; ++i)
        if (b.reqs[i]->out.stats)
          e = hipMemcpyAsync(b.reqs[i]->out.stats, d_stats[b.stream] + 2 * i, sizeof(uint64_t) * 2,
                             hipMemcpyDeviceToDevice, st);
      if (e != hipSuccess) s = device_error(ctx, e, "count copy");
    }
    if (s == LPA_OK) {
      e = hipEventCreateWithFlags(&b.done, hipEventDisableTiming);
      if (e == hipSuccess) e = hipEventRecord(b.done, st);
      if (e != hipSuccess) s = device_error(ctx, e, "batch event");
    }
    if (s != LPA_OK) {
      for (Request* r : b.reqs) finish(r, s);
      if (b.done) (void)hipEventDestroy(b.done);
      return;
    }
    for (Request* r : b.reqs) r->start_ns = t;
    inflight.push_back(std::move(b));
  }

  // Retire finished batches in order (caller holds mu).  Returns true if any.
  bool retire() {
    bool any = false;
    while (!inflight.empty()) {
      Batch& b = inflight.front();
      const hipError_t q = hipEventQuery(b.done);
      if (q == hipErrorNotReady) break;
      const int32_t st = q == hipSuccess ? LPA_OK : device_error(ctx, q, "batch execution");
      for (size_t i = 0; i < b.reqs.size(); ++i) {
        if (st == LPA_OK) {
          b.reqs[i]->n_fp64 = h_stats[b.stream][2 * i];
          b.reqs[i]->n_invalid = h_stats[b.stream][2 * i + 1];
        }
        finish(b.reqs[i], st);
      }
      (void)hipEventDestroy(b.done);
      inflight.erase(inflight.begin());
      any = true;
    }
    return any;
  }

  // Once the context has failed, frames not yet launched end with its error
  // (batches in flight still retire when their events complete).
  void fail_pending() {
    char msg[sizeof(g_last_error)];
    {
      std::lock_guard<std::mutex> g(ctx->fail_mu);
      std::snprintf(msg, sizeof(msg), "context failed after an earlier device error (%s)", ctx->fail_msg);
    }
    while (!waiting.empty() || !admitted.empty()) {
      std::deque<Request*>& q = waiting.empty() ? admitted : waiting;
      Request* r = q.front();
      q.pop_front();
      set_error(LPA_ERR_DEVICE, "%s", msg);
      finish(r, LPA_ERR_DEVICE);
    }
  }

  void run() {
    (void)hipSetDevice(ctx->device);
    std::unique_lock<std::mutex> lk(mu);
    while (true) {
      const bool retired = retire();
      if (ctx->failed.load()) fail_pending();
      admit();
      while (!admitted.empty() && (int)inflight.size() < kMaxInflight) launch();
      if (retired) cv_done.notify_all();
      if (stop && waiting.empty() && admitted.empty() && inflight.empty()) break;
      if (inflight.empty() && admitted.empty() && waiting.empty()) {
        cv.wait(lk);
      } else {
        // frames are running: check their completion often without holding the lock
        lk.unlock();
        std::this_thread::sleep_for(std::chrono::microseconds(50));
        lk.lock();
      }
    }
    cv_done.notify_all();
  }
};

// Frees what serve_init made (streams, count buffers, slots) and the scheduler.
static void serve_release(Scheduler* s) {
  s->pool.release();
  if (s->copy_stream) (void)hipStreamDestroy(s->copy_stream);
  for (hipStream_t st : s->compute)
    if (st) (void)hipStreamDestroy(st);
  for (int i = 0; i < 2; ++i) {
    if (s->d_stats[i]) (void)hipFree(s->d_stats[i]);
    if (s->h_stats[i]) (void)hipHostFree(s->h_stats[i]);
  }
  delete s;
}

lpa_status serve_init(lpa_ctx* ctx) {
  Scheduler* s = new (std::nothrow) Scheduler();
  if (!s) return set_error(LPA_ERR_OOM, "host allocation failed");
  s->ctx = ctx;
  if (const char* fa = std::getenv("LPA_TEST_FAIL_AFTER")) s->fail_after = std::strtoll(fa, nullptr, 10);
  hipError_t e = hipStreamCreateWithFlags(&s->copy_stream, hipStreamNonBlocking);
  for (int i = 0; e == hipSuccess && i < 2; ++i) e = hipStreamCreateWithFlags(&s->compute[i], hipStreamNonBlocking);
  const size_t sb = sizeof(uint64_t) * 2 * Scheduler::kMaxBatch;
  for (int i = 0; e == hipSuccess && i < 2; ++i) {
    e = hipMalloc(&s->d_stats[i], sb);
    if (e == hipSuccess) e = hipHostMalloc(&s->h_stats[i], sb, hipHostMallocDefault);
  }
  if (e != hipSuccess) {
    serve_release(s);
    return set_error(LPA_ERR_DEVICE, "scheduler set-up: %s", hipGetErrorString(e));
  }
  ctx->sched = s;
  s->worker = std::thread([s] { s->run(); });
  return LPA_OK;
}

void serve_shutdown(lpa_ctx* ctx) {
  Scheduler* s = ctx->sched;
  if (!s) return;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
  }
  s->cv.notify_all();
  if (s->worker.joinable()) s->worker.join();
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
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
    Scheduler* s = ctx->sched;
    Request* r = new (std::nothrow) Request();
    if (!r) return set_error(LPA_ERR_OOM, "host allocation failed");
    r->rig = rig;
    r->frame = *frame;
    r->params = *params;
    r->out = *out;
    r->arrival_ns = arrival_ns ? arrival_ns : now_ns();
    if (frame->memory == LPA_MEM_HOST) {
      const size_t es = frame->dtype == LPA_DTYPE_U16 ? 2 : 4;
      for (int i = 0; i < rig->n; ++i)
        r->raw_bytes += (es * rig->desc[i].width * rig->desc[i].height + 255) / 256 * 256;
    }
    {
      std::lock_guard<std::mutex> g(s->mu);
      if (s->waiting.size() >= Scheduler::kQueueCap) {
        delete r;
        return set_error(LPA_AGAIN, "admission queue full");
      }
      r->ticket = s->next_ticket++;
      *ticket = r->ticket;
      s->results[r->ticket] = lpa_result{LPA_NOT_READY, 0, r->arrival_ns, 0, 0, 0};
      s->waiting.push_back(r);
      ++s->pending;
    }
    s->cv.notify_all();
    return LPA_OK;
  } catch (...) {
    return set_error(LPA_ERR_INTERNAL, "unexpected exception");
  }
}

lpa_status lpa_poll(lpa_ctx* ctx, uint64_t ticket, lpa_result* out) {
  if (!ctx || !out) return set_error(LPA_ERR_INVALID_ARG, "context or result is NULL");
  Scheduler* s = ctx->sched;
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->results.find(ticket);
  if (it == s->results.end()) return set_error(LPA_ERR_INVALID_ARG, "unknown ticket %llu", (unsigned long long)ticket);
  *out = it->second;
  if (out->status == LPA_NOT_READY) return LPA_NOT_READY;
  s->results.erase(it);  // a terminal result is handed out once
  return LPA_OK;
}

lpa_status lpa_drain(lpa_ctx* ctx) {
  if (!ctx) return set_error(LPA_ERR_INVALID_ARG, "context is NULL");
  Scheduler* s = ctx->sched;
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_done.wait(lk, [s] { return s->pending == 0; });
  return ctx->failed.load() ? set_error(LPA_ERR_DEVICE, "context failed") : LPA_OK;
}

}  // extern "C"
