// lpa_host.hpp -- host-side state behind the C ABI (contexts, rigs, the
// autotuner and the serving scheduler).
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <atomic>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <set>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/lpa.h"
#include "lpa_internal.hpp"

namespace lpa {

struct Resolved {
  lpa_params p;
  double tau_inv, tau_fp64, gamma;
  double h[LPA_MAX_SCALES];
  // CALPA (mode == LPA_MODE_CALPA), defaults applied
  double grad_radius = 0, grad_h = 0, max_stretch = 1;
  int grad_order = 1;
  // support boxes cover radius * box_stretch (max_stretch for the steered fit)
  double box_stretch = 1;
};

// Class of a frame for tuning: everything that changes the kernel's cost per
// pixel, nothing that depends on the frame's data.  A frame's tuning choice
// depends only on its class, so its result does not depend on the other
// frames it is launched with.
struct TuneKey {
  int order, n_scales, n_sensors, src_kind;
  int radius_q;  // largest radius in 1/8 px
  int zoom_q;    // output-to-sensor scale in 1/16
  bool operator<(const TuneKey& o) const {
    const int a[6] = {order, n_scales, n_sensors, src_kind, radius_q, zoom_q};
    const int b[6] = {o.order, o.n_scales, o.n_sensors, o.src_kind, o.radius_q, o.zoom_q};
    for (int i = 0; i < 6; ++i)
      if (a[i] != b[i]) return a[i] < b[i];
    return false;
  }
};

struct TuneChoice {
  int tile_w = 16, tile_h = 16, occupancy = 0;
};

struct lpa_rig_fwd;

class Tuner {
 public:
  // Tile shape for a frame's class: the measured best if the class was tuned,
  // else 16 x 16.  Every candidate has 256 lanes, so batched launches can mix
  // classes.
  TuneChoice choose(const TuneKey& k) {
    TuneChoice c;
    if (!lookup(k, &c)) c = TuneChoice();
    return c;
  }
  void set(const TuneKey& k, TuneChoice c) {
    std::lock_guard<std::mutex> g(mu_);
    table_[k] = c;
  }
  bool lookup(const TuneKey& k, TuneChoice* c) {
    std::lock_guard<std::mutex> g(mu_);
    auto it = table_.find(k);
    if (it == table_.end()) return false;
    *c = it->second;
    return true;
  }
  static TuneKey key_of(const struct ::lpa_rig* rig, const Resolved& R, int src_kind);
  size_t size() {
    std::lock_guard<std::mutex> g(mu_);
    return table_.size();
  }
  std::map<TuneKey, TuneChoice> snapshot() {
    std::lock_guard<std::mutex> g(mu_);
    return table_;
  }

 private:
  std::mutex mu_;
  std::map<TuneKey, TuneChoice> table_;
};

// One reusable batch table: pinned host staging, device copy, the graph that
// copies it and runs the batch's kernels, and an event marking the end of its
// last use.
struct BatchSlot {
  void* h_buf = nullptr;
  void* d_buf = nullptr;
  int cap = 0;
  hipEvent_t done = nullptr;
  bool used = false;
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;     // kept with exec: its node handles name the nodes to update
  hipGraphNode_t fit_node = nullptr, refit_node = nullptr;
  int64_t sig[5] = {0, 0, 0, 0, 0};  // source kind, block, grid, capacity, raw float DN
  int lds = 0;                    // dynamic LDS of the fit node (float2 elements)
  int refit_lds = 0;              // dynamic LDS of the refit node (bytes)
  int refit_grid = 0;             // workgroups of the refit node
};

// Byte layout of a batch table of capacity cap.
struct BatchLayout {
  size_t frames_off, first_off, queue_off, copy_bytes, total_bytes;
  explicit BatchLayout(int cap) {
    frames_off = 256;
    first_off = frames_off + sizeof(LaunchK) * (size_t)cap;
    queue_off = (first_off + sizeof(int64_t) * (size_t)cap + 255) / 256 * 256;
    copy_bytes = first_off + sizeof(int64_t) * (size_t)cap;
    total_bytes = queue_off + 256;
  }
};

struct Scheduler;  // lpa_serve.cpp

}  // namespace lpa

struct lpa_ctx {
  int device = 0;
  int n_cu = 256;
  size_t budget = 0;
  std::atomic<size_t> used{0};
  std::atomic<bool> failed{false};
  std::mutex fail_mu;
  char fail_msg[256] = {0};  // message of the first device error
  lpa::Tuner tuner;
  // batch path: a ring of reusable tables, each with its graph
  std::mutex batch_mu;
  std::vector<lpa::BatchSlot> slots;
  int next_slot = 0;
  // serving
  lpa::Scheduler* sched = nullptr;
  // live rigs (destroyed with the context)
  std::mutex rigs_mu;
  std::set<lpa_rig*> rigs;
  // kernel timing (lpa_set_kernel_timing): per bracketed frame, events before
  // the fit, after the fit and after the refit (null: no refit launched)
  std::mutex timing_mu;
  bool timing = false;
  std::vector<std::array<hipEvent_t, 3>> timing_events;
};

struct lpa_rig {
  lpa_ctx* ctx = nullptr;
  int n = 0;
  lpa_sensor_desc desc[LPA_MAX_SENSORS];
  lpa::SensorK k[LPA_MAX_SENSORS];  // host copy of the resident constants
  lpa::SensorK* d_k = nullptr;       // device-resident constants
  size_t calib_bytes[LPA_MAX_SENSORS] = {0};  // budget charged for calibration planes
  // Pre-computed-weight tables, one per parameter class, built on first use
  // and kept until the rig is destroyed (a table may be read by queued work).
  struct Stencil {
    std::vector<double> key;
    void* d = nullptr;
    size_t bytes = 0;
  };
  std::mutex stencil_mu;
  std::vector<Stencil> stencils;
};

namespace lpa {

extern thread_local char g_last_error[512];
lpa_status set_error(lpa_status st, const char* fmt, ...);
lpa_status device_error(lpa_ctx* ctx, hipError_t e, const char* what);
lpa_status check_ctx(lpa_ctx* ctx);
lpa_status resolve_params(const lpa_params* p, Resolved* r);
lpa_status validate_frame(const lpa_rig* rig, const lpa_frame* f, bool need_device);
lpa_status validate_output(const lpa_params* p, const lpa_output* o);
// A launch descriptor for `frame` (its raw planes are what the FP64 refit
// reads; srcs / pitches are where the fit reads samples: the raw planes or
// pre-pass planes, null until the pre-pass has run).
lpa_status build_launch(const lpa_rig* rig, const Resolved& R, const lpa_frame* frame, const lpa_output* out,
                        int src_kind, const void* const* srcs, const int64_t* pitches, int tile_w, int tile_h,
                        LaunchK* K);
lpa_status build_launch_fit(const lpa_rig* rig, const Resolved& R, const lpa_frame* frame, const lpa_output* out,
                            int src_kind, const void* const* srcs, const int64_t* pitches, int pref_w, int pref_h,
                            LaunchK* K);
// Stream-ordered scratch; `charge` counts it against the context's HBM budget
// (the serving scheduler charges a frame's whole footprint at admission).
lpa_status alloc_async(lpa_ctx* ctx, size_t bytes, hipStream_t st, void** p, bool charge = true);
void free_async(lpa_ctx* ctx, void* p, size_t bytes, hipStream_t st, bool charge = true);
// Allocates a frame's pre-pass planes (stream-ordered) and enqueues the
// pre-pass of every sensor (batches carve their planes from one allocation
// and their graph fills them).
lpa_status run_prepass(lpa_rig* rig, const lpa_frame* f, bool to_f16, hipStream_t st, void** planes,
                       size_t* plane_bytes, const void** srcs, int64_t* pitches, bool charge = true);
// Pre-computed-weight table of a launch (lpa_stencil.cpp): checks that every
// sensor map and the output map are translations, then returns the rig's
// cached device table for the launch's radii and windows, building it on
// first use.
lpa_status stencil_table(lpa_rig* rig, const Resolved& R, const LaunchK& K, const StencilTable** out);
void stencil_free(lpa_rig* rig);

// Runtime pieces owned by a context (scheduler threads, batch tables).
lpa_status ctx_init_runtime(lpa_ctx* ctx);
void ctx_shutdown_runtime(lpa_ctx* ctx);

// Launch a prepared batch (descriptors already built, planes already made) on
// `stream` through a slot's captured graph.  Thread-safe.
// Frames whose outputs ask for counts get a per-tile count buffer (8 bytes per
// tile) for the launch; `charge` counts it against the budget.
lpa_status launch_batch(lpa_ctx* ctx, const std::vector<LaunchK>& ks, int src_kind, hipStream_t stream,
                        bool charge = true);
// Build descriptors for a list of frames (validating each) and run the
// pre-pass where the storage form needs one; plane allocations are returned
// for the caller to free (stream-ordered) after the launch.
struct PlaneAlloc {
  void* p;
  size_t bytes;
};
lpa_status prepare_frames(lpa_ctx* ctx, int n, lpa_rig* const* rigs, const lpa_frame* frames,
                          const lpa_params* params, const lpa_output* outs, hipStream_t stream,
                          std::vector<LaunchK>* ks, int* src_kind, std::vector<PlaneAlloc>* planes,
                          bool charge = true);
// Whether a frame can join a batch: some 256-lane tile shape stages its
// windows (LPA_ERR_UNSUPPORTED with the reason otherwise).
lpa_status check_batchable(const lpa_rig* rig, const Resolved& R, const lpa_frame* frame, const lpa_output* out);
// Device address of the allocation-free entry point's static scratch on the
// current device (lpa_noalloc.cpp); called by lpa_create_ctx.
lpa_status noalloc_init_device(int device);
lpa_status serve_init(lpa_ctx* ctx);
void serve_shutdown(lpa_ctx* ctx);

// Kernel timing of one frame (lpa_set_kernel_timing): when the context's
// timing is on, mark(0) before the fit launch, mark(1) after it, mark(2)
// after the refit launch; commit() hands the events to the context.  Events
// of a frame that is not committed (an error path) are destroyed.
class KernelBracket {
 public:
  KernelBracket(lpa_ctx* ctx, hipStream_t hs);
  ~KernelBracket();
  void mark(int i);
  void commit(bool refit_launched);

 private:
  lpa_ctx* ctx_;
  hipStream_t hs_;
  std::array<hipEvent_t, 3> ev_{};
  bool on_ = false;
};
void timing_clear_locked(lpa_ctx* ctx);

}  // namespace lpa
