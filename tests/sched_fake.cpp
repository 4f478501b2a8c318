// The serving scheduler's policy (SchedCore, lpa_sched.hpp) driven by a fake
// executor on the CPU, for runs under ThreadSanitizer and AddressSanitizer.
//
// The fake device is a thread that completes launched batches after a
// simulated duration; client threads submit and poll concurrently.  The fake
// checks the scheduler's contract as it is called:
//   * every executor call but thread_start runs on the scheduler thread;
//   * frames are admitted in ticket order, and the budget holds at admission;
//   * a launch has 1..64 frames of one batch key, at most 2 launches are in
//     flight, on different streams, and none starts after the context failed;
//   * each frame and each batch is released exactly once.
// The clients check every ticket's result: handed out once, the expected
// status and counts, ordered timestamps.  Prints "ok <scenario>" per
// scenario; any failed check prints "FAIL ..." and exits non-zero.
//
// usage: sched_fake <mixed|fail|queue_full> [seed]
#include <atomic>
#include <cinttypes>
#include <cstdarg>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <random>
#include <set>
#include <string>
#include <thread>
#include <vector>

#include "../paper_1308_4908_amd/csrc/lpa_sched.hpp"

using lpa::SchedCore;

static std::mutex g_fail_mu;
static std::vector<std::string> g_fail;

static void fail(const char* fmt, ...) __attribute__((format(printf, 1, 2)));
static void fail(const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  std::lock_guard<std::mutex> g(g_fail_mu);
  if (g_fail.size() < 50) g_fail.push_back(buf);
}

#define CHECK(c, ...)            \
  do {                           \
    if (!(c)) fail(__VA_ARGS__); \
  } while (0)

struct FakeJob {
  int id = -1;
  size_t bytes = 0;
  uint64_t key = 0;
  int work_us = 0;
  bool copy_fails = false;
};

// A launched batch as the fake device sees it.
struct DevBatch {
  std::atomic<int> state{0};  // 0 running, 1 done
  int work_us = 0;
};

struct FakeBatch {
  std::shared_ptr<DevBatch> dev;
  std::vector<int> ids;
  int stream = -1;
};

// The simulated device: completes batches in launch order.  A closed gate
// holds every batch until it opens.
class FakeDevice {
 public:
  FakeDevice() : thr_([this] { loop(); }) {}
  ~FakeDevice() {
    {
      std::lock_guard<std::mutex> g(mu_);
      stop_ = true;
      gate_ = true;
    }
    cv_.notify_all();
    thr_.join();
  }
  void enqueue(std::shared_ptr<DevBatch> b) {
    {
      std::lock_guard<std::mutex> g(mu_);
      q_.push_back(std::move(b));
    }
    cv_.notify_all();
  }
  void set_gate(bool open) {
    {
      std::lock_guard<std::mutex> g(mu_);
      gate_ = open;
    }
    cv_.notify_all();
  }

 private:
  void loop() {
    std::unique_lock<std::mutex> lk(mu_);
    while (true) {
      cv_.wait(lk, [this] { return stop_ || (gate_ && !q_.empty()); });
      if (q_.empty() && stop_) return;
      std::shared_ptr<DevBatch> b = q_.front();
      q_.pop_front();
      lk.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(b->work_us));
      b->state.store(1, std::memory_order_release);
      lk.lock();
    }
  }
  std::mutex mu_;
  std::condition_variable cv_;
  std::deque<std::shared_ptr<DevBatch>> q_;
  bool gate_ = true, stop_ = false;
  std::thread thr_;
};

struct FakeExec {
  using Job = FakeJob;
  using Batch = FakeBatch;

  FakeDevice* dev = nullptr;
  std::atomic<size_t>* used = nullptr;
  size_t budget = 0;
  int64_t fail_after = 0;  // the n-th launch fails (0: never)
  // scheduler-thread state (checked to be touched only there)
  std::thread::id sched_tid;
  std::atomic<bool> have_tid{false};
  std::atomic<bool> failed_{false};
  int64_t launches = 0;
  int inflight = 0;
  bool busy[2] = {false, false};
  std::set<int> live_jobs;            // admitted, not released
  std::vector<int> admitted_order;    // ids in admission order
  std::set<int> released;
  std::mutex report_mu;
  std::string last_report;
  int last_status = 0;

  void on_sched(const char* what) {
    CHECK(have_tid.load() && std::this_thread::get_id() == sched_tid, "%s off the scheduler thread", what);
  }
  void thread_start() {
    sched_tid = std::this_thread::get_id();
    have_tid.store(true);
  }
  bool failed() {
    on_sched("failed");
    return failed_.load();
  }
  void failure_message(char* buf, size_t n) {
    on_sched("failure_message");
    std::snprintf(buf, n, "injected");
  }
  void report(int32_t status, const char* msg) {
    std::lock_guard<std::mutex> g(report_mu);
    last_status = status;
    last_report = msg;
  }
  size_t footprint(const Job& j) {
    on_sched("footprint");
    return j.bytes;
  }
  uint64_t batch_key(const Job& j) {
    on_sched("batch_key");
    return j.key;
  }
  int32_t admit(Job& j) {
    on_sched("admit");
    CHECK(used->load() <= budget, "budget exceeded at admission of %d: %zu > %zu", j.id, used->load(), budget);
    CHECK(live_jobs.insert(j.id).second, "frame %d admitted twice", j.id);
    admitted_order.push_back(j.id);
    return j.copy_fails ? LPA_ERR_INTERNAL : LPA_OK;
  }
  int32_t launch(Job* const* jobs, int n, int stream, Batch& b) {
    on_sched("launch");
    CHECK(!failed_.load(), "launch after the context failed");
    CHECK(n >= 1 && n <= SchedCore<FakeExec>::kMaxBatch, "batch of %d frames", n);
    CHECK(stream == 0 || stream == 1, "stream %d", stream);
    CHECK(inflight < SchedCore<FakeExec>::kMaxInflight, "%d batches already in flight", inflight);
    CHECK(!busy[stream & 1], "stream %d busy", stream);
    b.stream = stream;
    int work = 20;
    for (int i = 0; i < n; ++i) {
      CHECK(jobs[i]->key == jobs[0]->key, "mixed keys in one batch");
      CHECK(live_jobs.count(jobs[i]->id) == 1, "frame %d launched without admission", jobs[i]->id);
      b.ids.push_back(jobs[i]->id);
      work += jobs[i]->work_us / 4;
    }
    if (fail_after > 0 && ++launches >= fail_after) {
      failed_.store(true);
      return LPA_ERR_DEVICE;
    }
    ++inflight;
    busy[stream & 1] = true;
    b.dev = std::make_shared<DevBatch>();
    b.dev->work_us = work;
    dev->enqueue(b.dev);
    return LPA_OK;
  }
  int32_t query(Batch& b) {
    on_sched("query");
    return b.dev->state.load(std::memory_order_acquire) ? LPA_OK : LPA_NOT_READY;
  }
  void counts(const Batch& b, int i, uint64_t* n_fp64, uint64_t* n_invalid) {
    on_sched("counts");
    *n_fp64 = 3u * (uint64_t)b.ids[i] + 1u;
    *n_invalid = (uint64_t)b.ids[i] % 5u;
  }
  void release(Job& j) {
    on_sched("release(job)");
    CHECK(released.insert(j.id).second, "frame %d released twice", j.id);
    live_jobs.erase(j.id);
  }
  void release(Batch& b) {
    on_sched("release(batch)");
    if (b.dev) {  // a launched batch (a failed launch enqueued nothing)
      CHECK(b.stream == 0 || b.stream == 1, "released batch without a stream");
      --inflight;
      busy[b.stream & 1] = false;
      b.dev.reset();
    }
  }
};

struct Expect {
  int id;
  uint64_t ticket;
  int32_t status;  // expected terminal status (LPA_OK, ...) or 99: OK or device error
};

// Polls `mine` until every ticket is terminal; checks each result.
static void poll_all(SchedCore<FakeExec>& core, std::vector<Expect>& mine, std::mt19937& rng, int* n_dev_err) {
  std::vector<bool> done(mine.size(), false);
  size_t left = mine.size();
  while (left) {
    for (size_t k = 0; k < mine.size(); ++k) {
      if (done[k] || (rng() & 3) == 0) continue;
      lpa_result r{};
      const int32_t s = core.poll(mine[k].ticket, &r);
      if (s == LPA_NOT_READY) {
        CHECK(r.status == LPA_NOT_READY, "NOT_READY with status %d", r.status);
        continue;
      }
      CHECK(s == LPA_OK, "poll of %" PRIu64 " returned %d", mine[k].ticket, s);
      done[k] = true;
      --left;
      const Expect& e = mine[k];
      if (e.status == 99) {
        CHECK(r.status == LPA_OK || r.status == LPA_ERR_DEVICE, "frame %d: status %d", e.id, r.status);
        if (r.status == LPA_ERR_DEVICE) ++*n_dev_err;
      } else {
        CHECK(r.status == e.status, "frame %d: status %d, expected %d", e.id, r.status, e.status);
      }
      if (r.status == LPA_OK) {
        CHECK(r.n_fp64 == 3u * (uint64_t)e.id + 1u && r.n_invalid == (uint64_t)e.id % 5u, "frame %d: counts", e.id);
        CHECK(r.batch_size >= 1 && r.batch_size <= 64, "frame %d: batch size %d", e.id, r.batch_size);
        CHECK(r.t_arrival_ns <= r.t_admit_ns && r.t_admit_ns <= r.t_start_ns && r.t_start_ns <= r.t_done_ns,
              "frame %d: timestamps out of order", e.id);
      }
      lpa_result again{};
      CHECK(core.poll(e.ticket, &again) == LPA_ERR_INVALID_ARG, "ticket %" PRIu64 " handed out twice", e.ticket);
    }
    std::this_thread::sleep_for(std::chrono::microseconds(100));
  }
}

struct Setup {
  FakeDevice dev;
  std::atomic<size_t> used{0};
  FakeExec exec;
  std::unique_ptr<SchedCore<FakeExec>> core;
  Setup(size_t budget, size_t resident, int64_t fail_after) {
    used.store(resident);
    exec.dev = &dev;
    exec.used = &used;
    exec.budget = budget;
    exec.fail_after = fail_after;
    core.reset(new SchedCore<FakeExec>(exec, used, budget));
    core->start();
  }
};

// Admission order is ticket order (the queue is FIFO).
static void check_fifo(const FakeExec& ex, const std::map<int, uint64_t>& ticket_of) {
  uint64_t last = 0;
  for (int id : ex.admitted_order) {
    auto it = ticket_of.find(id);
    CHECK(it != ticket_of.end(), "admitted frame %d was never submitted", id);
    if (it == ticket_of.end()) continue;
    CHECK(it->second > last, "frame %d admitted out of order", id);
    last = it->second;
  }
}

static int scenario_mixed(unsigned seed) {
  const size_t budget = 10000, resident = 1000;
  Setup S(budget, resident, 0);
  constexpr int kClients = 4, kPer = 400;
  std::mutex map_mu;
  std::map<int, uint64_t> ticket_of;
  std::vector<std::thread> clients;
  std::atomic<int> n_ok{0};
  for (int c = 0; c < kClients; ++c) {
    clients.emplace_back([&, c] {
      std::mt19937 rng(seed * 7919u + (unsigned)c);
      std::vector<Expect> mine;
      uint64_t key = rng() & 1;
      for (int k = 0; k < kPer; ++k) {
        FakeJob j;
        j.id = c * kPer + k;
        if (rng() % 10 == 0) key ^= 1;
        j.key = key;
        j.bytes = 1 + rng() % 3000;
        int32_t expect = LPA_OK;
        if (rng() % 50 == 0) {
          j.bytes = budget - resident + 1 + rng() % 500;  // never fits beside the resident bytes
          expect = LPA_ERR_OOM;
        } else if (rng() % 100 == 0) {
          j.copy_fails = true;
          expect = LPA_ERR_INTERNAL;
        }
        j.work_us = (int)(rng() % 200);
        const int id = j.id;
        uint64_t t = 0;
        int32_t s;
        while ((s = S.core->submit(FakeJob(j), 0, &t)) == LPA_AGAIN) std::this_thread::sleep_for(std::chrono::microseconds(200));
        CHECK(s == LPA_OK, "submit returned %d", s);
        {
          std::lock_guard<std::mutex> g(map_mu);
          ticket_of[id] = t;
        }
        mine.push_back({id, t, expect});
        if (rng() % 8 == 0) std::this_thread::sleep_for(std::chrono::microseconds(rng() % 300));
      }
      int dev_err = 0;
      poll_all(*S.core, mine, rng, &dev_err);
      CHECK(dev_err == 0, "device errors without a failure");
      n_ok.fetch_add((int)mine.size());
    });
  }
  for (auto& t : clients) t.join();
  S.core->drain();
  CHECK(n_ok.load() == kClients * kPer, "polled %d results", n_ok.load());
  CHECK(S.core->results_held() == 0, "%zu results left after every ticket was polled", S.core->results_held());
  S.core->stop();
  CHECK(S.used.load() == resident, "charge %zu after drain, expected %zu", S.used.load(), resident);
  CHECK(S.exec.released.size() == (size_t)(kClients * kPer), "released %zu frames", S.exec.released.size());
  CHECK(S.exec.inflight == 0, "%d batches never released", S.exec.inflight);
  check_fifo(S.exec, ticket_of);
  return 0;
}

static int scenario_fail(unsigned seed) {
  const size_t budget = 1 << 20;
  Setup S(budget, 0, 5);
  constexpr int kClients = 2, kPer = 300;
  std::map<int, uint64_t> ticket_of;
  std::mutex map_mu;
  std::atomic<int> dev_errs{0};
  std::vector<std::thread> clients;
  for (int c = 0; c < kClients; ++c) {
    clients.emplace_back([&, c] {
      std::mt19937 rng(seed * 31u + (unsigned)c);
      std::vector<Expect> mine;
      for (int k = 0; k < kPer; ++k) {
        FakeJob j;
        j.id = c * kPer + k;
        j.bytes = 1000;
        j.work_us = 200;
        uint64_t t = 0;
        const int32_t s = S.core->submit(FakeJob(j), 0, &t);
        CHECK(s == LPA_OK, "submit returned %d", s);
        {
          std::lock_guard<std::mutex> g(map_mu);
          ticket_of[j.id] = t;
        }
        mine.push_back({j.id, t, 99});
        if (k % 16 == 0) std::this_thread::sleep_for(std::chrono::microseconds(500));
      }
      int dev_err = 0;
      poll_all(*S.core, mine, rng, &dev_err);
      dev_errs.fetch_add(dev_err);
    });
  }
  for (auto& t : clients) t.join();
  S.core->drain();
  CHECK(S.exec.failed_.load(), "the injected failure never happened");
  CHECK(dev_errs.load() > 0, "no frame ended with the device error");
  {
    std::lock_guard<std::mutex> g(S.exec.report_mu);
    CHECK(S.exec.last_status == LPA_ERR_DEVICE && S.exec.last_report.find("injected") != std::string::npos,
          "last report: %d %s", S.exec.last_status, S.exec.last_report.c_str());
  }
  S.core->stop();
  CHECK(S.used.load() == 0, "charge %zu after drain", S.used.load());
  CHECK(S.exec.released.size() == (size_t)(kClients * kPer), "released %zu frames", S.exec.released.size());
  check_fifo(S.exec, ticket_of);
  return 0;
}

static int scenario_queue_full(unsigned seed) {
  const size_t budget = 10000;
  Setup S(budget, 0, 0);
  S.dev.set_gate(false);  // nothing completes: the queue fills
  std::mt19937 rng(seed);
  std::vector<Expect> mine;
  int again = 0;
  for (int k = 0; k < 1100; ++k) {
    FakeJob j;
    j.id = k;
    j.bytes = 6000;  // one frame in flight at a time
    uint64_t t = 0;
    const int32_t s = S.core->submit(FakeJob(j), 0, &t);
    if (s == LPA_AGAIN) {
      ++again;
      continue;
    }
    CHECK(s == LPA_OK, "submit returned %d", s);
    mine.push_back({k, t, LPA_OK});
  }
  CHECK(again > 0, "the queue never reported full");
  CHECK(mine.size() >= SchedCore<FakeExec>::kQueueCap && mine.size() <= SchedCore<FakeExec>::kQueueCap + 3,
        "%zu frames accepted", mine.size());
  S.dev.set_gate(true);
  int dev_err = 0;
  poll_all(*S.core, mine, rng, &dev_err);
  S.core->drain();
  S.core->stop();
  CHECK(S.used.load() == 0, "charge %zu after drain", S.used.load());
  return 0;
}

int main(int argc, char** argv) {
  if (argc < 2) {
    std::fprintf(stderr, "usage: %s <mixed|fail|queue_full> [seed]\n", argv[0]);
    return 2;
  }
  const unsigned seed = argc > 2 ? (unsigned)std::strtoul(argv[2], nullptr, 10) : 1u;
  const std::string sc = argv[1];
  if (sc == "mixed") scenario_mixed(seed);
  else if (sc == "fail") scenario_fail(seed);
  else if (sc == "queue_full") scenario_queue_full(seed);
  else {
    std::fprintf(stderr, "unknown scenario %s\n", sc.c_str());
    return 2;
  }
  if (!g_fail.empty()) {
    for (const std::string& f : g_fail) std::printf("FAIL %s\n", f.c_str());
    return 1;
  }
  std::printf("ok %s\n", sc.c_str());
  return 0;
}
