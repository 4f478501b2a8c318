// lpa_sched.hpp -- the serving scheduler's policy (admission, batching,
// completion), apart from the device it drives.
//
// SchedCore<Exec> owns the queues, the tickets and their results, and the
// charge against the byte budget.  Exec does everything that touches the
// device; lpa_serve.cpp gives the HIP one, and a CPU test gives a fake one
// (run under ThreadSanitizer).  Exec provides:
//   typename Exec::Job    what one frame needs on the device
//   typename Exec::Batch  one launch's device state (its completion event)
//   size_t   footprint(const Job&)     bytes charged at admission
//   int32_t  admit(Job&)               starts the frame's copy to the device
//   uint64_t batch_key(const Job&)     frames with equal keys may share a launch
//   int32_t  launch(Job* const* jobs, int n, int stream, Batch&)
//                                      enqueues one launch over n frames on
//                                      compute stream `stream` (0 or 1)
//   int32_t  query(Batch&)             LPA_NOT_READY, LPA_OK or an error
//   void     counts(const Batch&, int i, uint64_t* n_fp64, uint64_t* n_invalid)
//   void     release(Job&)             the frame has ended: its copy slot returns
//   void     release(Batch&)           the batch has ended (or failed to launch)
//   bool     failed()                  the device context has failed
//   void     failure_message(char*, size_t)  what made it fail
//   void     report(int32_t status, const char* msg)  the caller's error record
//   void     thread_start()            run first on the scheduler thread
//
// Policy:
//   admission  FIFO: the oldest waiting frame is admitted once the budget
//              holds its footprint beside what is already charged; while it
//              does not fit, the frames behind it wait too.  A frame that does
//              not fit when nothing of the scheduler's is charged never will:
//              it ends with LPA_ERR_OOM.
//   batching   every admitted frame joins the next launch (at most kMaxBatch,
//              the longest prefix of equal batch keys), with at most
//              kMaxInflight launches in flight, each on its own stream.
//   completion launches retire in launch order; their frames take their
//              counts, their timestamps and their status.
//   failure    once the context has failed, nothing more is admitted or
//              launched: frames not yet launched end with LPA_ERR_DEVICE
//              (launches in flight still retire).
#pragma once

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <cstdio>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <utility>
#include <vector>

#include "../../include/lpa.h"

namespace lpa {

inline int64_t sched_now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

template <class Exec>
class SchedCore {
 public:
  static constexpr size_t kQueueCap = 1024;
  static constexpr int kMaxInflight = 2;
  static constexpr int kMaxBatch = 64;

  // `used` is the context-wide charge (other holders, such as resident
  // calibration planes, charge it too); `budget` its limit.
  SchedCore(Exec& exec, std::atomic<size_t>& used, size_t budget) : exec_(exec), used_(used), budget_(budget) {}
  SchedCore(const SchedCore&) = delete;
  SchedCore& operator=(const SchedCore&) = delete;
  ~SchedCore() { stop(); }

  void start() {
    worker_ = std::thread([this] {
      exec_.thread_start();
      run();
    });
  }

  // Finishes every submitted frame, then ends the scheduler thread.
  void stop() {
    {
      std::lock_guard<std::mutex> g(mu_);
      stop_ = true;
    }
    cv_.notify_all();
    if (worker_.joinable()) worker_.join();
  }

  // Queues a frame.  LPA_AGAIN if kQueueCap frames already wait.
  int32_t submit(typename Exec::Job&& job, int64_t arrival_ns, uint64_t* ticket) {
    Request* r = new (std::nothrow) Request{};
    if (!r) return LPA_ERR_OOM;
    r->job = std::move(job);
    r->arrival_ns = arrival_ns ? arrival_ns : sched_now_ns();
    {
      std::lock_guard<std::mutex> g(mu_);
      if (waiting_.size() >= kQueueCap) {
        delete r;
        return LPA_AGAIN;
      }
      r->ticket = next_ticket_++;
      *ticket = r->ticket;
      results_[r->ticket] = lpa_result{LPA_NOT_READY, 0, r->arrival_ns, 0, 0, 0, 0, 0};
      waiting_.push_back(r);
      ++pending_;
    }
    cv_.notify_all();
    return LPA_OK;
  }

  // LPA_NOT_READY (with the timestamps so far), or the terminal result, which
  // is handed out once: the ticket is then forgotten.  LPA_ERR_INVALID_ARG
  // for a ticket that is unknown or already handed out.
  int32_t poll(uint64_t ticket, lpa_result* out) {
    std::lock_guard<std::mutex> g(mu_);
    auto it = results_.find(ticket);
    if (it == results_.end()) return LPA_ERR_INVALID_ARG;
    *out = it->second;
    if (out->status == LPA_NOT_READY) return LPA_NOT_READY;
    results_.erase(it);
    return LPA_OK;
  }

  // Blocks until every submitted frame has ended.
  void drain() {
    std::unique_lock<std::mutex> lk(mu_);
    cv_done_.wait(lk, [this] { return pending_ == 0; });
  }

  size_t results_held() {
    std::lock_guard<std::mutex> g(mu_);
    return results_.size();
  }

 private:
  struct Request {
    uint64_t ticket;
    typename Exec::Job job;
    int64_t arrival_ns, admit_ns, start_ns, done_ns;
    size_t reserved;  // bytes charged at admission
    int32_t batch_size;
    uint64_t n_fp64, n_invalid;
  };
  struct Batch {
    std::vector<Request*> reqs;
    typename Exec::Batch dev;
    int stream = 0;
  };

  void report(int32_t status, const char* fmt, size_t a, size_t b, size_t c) {
    char msg[256];
    std::snprintf(msg, sizeof(msg), fmt, a, b, c);
    exec_.report(status, msg);
  }

  // The frame has ended (caller holds mu_).
  void finish(Request* r, int32_t status) {
    r->done_ns = sched_now_ns();
    lpa_result res;
    res.status = status;
    res.batch_size = r->batch_size;
    res.t_arrival_ns = r->arrival_ns;
    res.t_admit_ns = r->admit_ns;
    res.t_start_ns = r->start_ns;
    res.t_done_ns = r->done_ns;
    res.n_fp64 = r->n_fp64;
    res.n_invalid = r->n_invalid;
    results_[r->ticket] = res;
    exec_.release(r->job);  // the launch that read its slot has completed
    used_.fetch_sub(r->reserved);
    delete r;
    --pending_;
    // every terminal path (completion, rejection at admission, launch
    // failure) must wake drain(), which waits for pending_ == 0
    cv_done_.notify_all();
  }

  // Admit waiting frames in order while the budget allows (caller holds mu_).
  void admit() {
    while (!waiting_.empty() && !exec_.failed()) {
      Request* r = waiting_.front();
      const size_t need = exec_.footprint(r->job);
      if (used_.load() + need > budget_) {
        // frames in flight will return their memory; without any, what the
        // context holds stays, and this frame never fits beside it
        if (!admitted_.empty() || !inflight_.empty()) return;
        waiting_.pop_front();
        report(LPA_ERR_OOM, "frame needs %zu bytes; %zu of the budget of %zu are held", need, used_.load(),
               budget_);
        finish(r, LPA_ERR_OOM);
        continue;
      }
      used_.fetch_add(need);
      r->reserved = need;
      waiting_.pop_front();
      r->admit_ns = sched_now_ns();
      const int32_t s = exec_.admit(r->job);
      if (s != LPA_OK) {
        finish(r, s);
        continue;
      }
      admitted_.push_back(r);
    }
  }

  // Launch admitted frames as one batch (caller holds mu_, and fewer than
  // kMaxInflight batches are in flight).
  void launch() {
    const int n = (int)std::min<size_t>(admitted_.size(), kMaxBatch);
    const uint64_t key = exec_.batch_key(admitted_[0]->job);
    int take = 1;
    while (take < n && exec_.batch_key(admitted_[take]->job) == key) ++take;
    Batch b;
    b.reqs.assign(admitted_.begin(), admitted_.begin() + take);
    admitted_.erase(admitted_.begin(), admitted_.begin() + take);
    // the stream the batch in flight (if any) does not use
    b.stream = (!inflight_.empty() && inflight_.front().stream == 0) ? 1 : 0;
    std::vector<typename Exec::Job*> jobs;
    jobs.reserve(take);
    for (Request* r : b.reqs) {
      jobs.push_back(&r->job);
      r->batch_size = take;
    }
    const int64_t t = sched_now_ns();
    const int32_t s = exec_.launch(jobs.data(), take, b.stream, b.dev);
    if (s != LPA_OK) {
      for (Request* r : b.reqs) finish(r, s);
      exec_.release(b.dev);
      return;
    }
    for (Request* r : b.reqs) r->start_ns = t;
    inflight_.push_back(std::move(b));
  }

  // Retire finished batches in launch order (caller holds mu_).
  bool retire() {
    bool any = false;
    while (!inflight_.empty()) {
      Batch& b = inflight_.front();
      const int32_t q = exec_.query(b.dev);
      if (q == LPA_NOT_READY) break;
      for (size_t i = 0; i < b.reqs.size(); ++i) {
        if (q == LPA_OK) exec_.counts(b.dev, (int)i, &b.reqs[i]->n_fp64, &b.reqs[i]->n_invalid);
        finish(b.reqs[i], q);
      }
      exec_.release(b.dev);
      inflight_.pop_front();
      any = true;
    }
    return any;
  }

  // Once the context has failed, frames not yet launched end with its error.
  void fail_pending() {
    if (waiting_.empty() && admitted_.empty()) return;
    char why[256], msg[384];
    exec_.failure_message(why, sizeof(why));
    std::snprintf(msg, sizeof(msg), "context failed after an earlier device error (%s)", why);
    while (!waiting_.empty() || !admitted_.empty()) {
      std::deque<Request*>& q = waiting_.empty() ? admitted_ : waiting_;
      Request* r = q.front();
      q.pop_front();
      exec_.report(LPA_ERR_DEVICE, msg);
      finish(r, LPA_ERR_DEVICE);
    }
  }

  void run() {
    std::unique_lock<std::mutex> lk(mu_);
    while (true) {
      const bool retired = retire();
      if (!exec_.failed()) {
        admit();
        while (!admitted_.empty() && (int)inflight_.size() < kMaxInflight && !exec_.failed()) launch();
      }
      // a failure (here or in an earlier iteration) ends what is not launched
      if (exec_.failed()) fail_pending();
      if (retired) cv_done_.notify_all();
      if (stop_ && waiting_.empty() && admitted_.empty() && inflight_.empty()) break;
      if (inflight_.empty() && admitted_.empty() && waiting_.empty()) {
        cv_.wait(lk);
      } else {
        // frames are running: check their completion often, without the lock
        lk.unlock();
        std::this_thread::sleep_for(std::chrono::microseconds(50));
        lk.lock();
      }
    }
    cv_done_.notify_all();
  }

  Exec& exec_;
  std::atomic<size_t>& used_;
  const size_t budget_;
  std::mutex mu_;
  std::condition_variable cv_;       // wakes the scheduler thread
  std::condition_variable cv_done_;  // wakes drain()
  std::deque<Request*> waiting_;     // submitted, not admitted
  std::deque<Request*> admitted_;    // admitted, not launched
  std::deque<Batch> inflight_;
  std::unordered_map<uint64_t, lpa_result> results_;
  uint64_t next_ticket_ = 1;
  size_t pending_ = 0;  // submitted and not ended
  bool stop_ = false;
  std::thread worker_;
};

}  // namespace lpa
