/*
 * lpa.h -- C ABI of the MI355X (gfx950) library for multi-sensor HDR video
 * reconstruction by local polynomial approximation (LPA) with ICI window
 * selection, after Kronander, Gustavson, Bonnet, Ynnerman and Unger, "A
 * Unified Framework for Multi-Sensor HDR Video Reconstruction" (arXiv
 * 1308.4908).
 *
 * What one reconstruction computes, per output pixel j and colour channel c:
 *   - every raw CFA sample y of every sensor s is turned into a radiance
 *     estimate f = (y - b_s) / (g_s n_s) (Sec. 6, eq. Efsi) and a variance
 *     estimate (g_s^2 n_s f + Var r_s) / (g_s n_s)^2 (Sec. 6.1,
 *     eq. varianceestiamte; shot term clamped at 0); samples with
 *     y >= saturation are dropped (end of Sec. 6.1);
 *   - the sample sits at X = T_s(x) on the reference plane (Sec. 4.2), the
 *     output pixel at X_j = O(u, v) (arbitrary output grid, Sec. 3);
 *   - for each window radius r_m (ascending) the order-M local polynomial
 *     (Sec. 5.1) is fitted by weighted least squares, eq. (wlsqe), with weight
 *     K(|X - X_j|) / sigma^2, K(d) = exp(-d^2/h) - exp(-r^2/h) on d < r
 *     (isotropic Gaussian window of Sec. 5.3.1, truncated to vanish at r);
 *     a fit is valid when its support has at least as many samples as basis
 *     terms and the smallest pivot of the equilibrated normal matrix is at
 *     least tau_inv (the "invertible" rule of Sec. 5.3.1 made numeric);
 *   - intersection of confidence intervals (ICI) picks the radius: intervals
 *     C0 +- gamma * sd(C0) of the valid radii are intersected in ascending
 *     order and the last radius with a non-empty intersection is kept (the
 *     LPA-ICI rule of Goldenshluger-Nemirovski / Katkovnik; not in the paper);
 *   - if no radius is valid at order M the same supports are refitted at
 *     order M-1, ..., 0; if none is valid the output is NaN.
 *   The output is C0 per channel, in photo-electrons per unit exposure.
 *
 * Conventions: sensor pixel centres are at integer (x = column, y = row);
 * affine maps are [a0 a1 a2; a3 a4 a5]: X = a0 x + a1 y + a2,
 * Y = a3 x + a4 y + a5.  Radii and h are in reference-plane units.
 *
 * Errors: every call returns an lpa_status.  Arguments are validated before
 * anything is enqueued; on an error nothing is enqueued and outputs are left
 * untouched.  lpa_last_error() gives a thread-local message.  No C++
 * exception crosses this interface.  After a device error the context is
 * sticky-failed: every call on it returns LPA_ERR_DEVICE until it is
 * destroyed.
 */
#ifndef LPA_H
#define LPA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LPA_MAX_SENSORS 8
#define LPA_MAX_SCALES 8

typedef int32_t lpa_status;
enum {
  LPA_OK = 0,
  LPA_NOT_READY = 1,        /* lpa_poll: the frame is not finished yet          */
  LPA_AGAIN = 2,            /* lpa_submit: the admission queue is full          */
  LPA_ERR_INVALID_ARG = -1, /* argument failed validation; nothing enqueued    */
  LPA_ERR_OOM = -2,         /* device memory or HBM budget exhausted            */
  LPA_ERR_DEVICE = -3,      /* HIP runtime / device error (context now failed) */
  LPA_ERR_UNSUPPORTED = -4, /* valid request the library does not run           */
  LPA_ERR_INTERNAL = -5
};

enum { LPA_CFA_RGGB = 0, LPA_CFA_BGGR = 1, LPA_CFA_GRBG = 2, LPA_CFA_GBRG = 3 };
enum { LPA_DTYPE_U16 = 0, LPA_DTYPE_F32 = 1 }; /* raw sample type (F32: DN as float, tests) */
enum { LPA_MEM_DEVICE = 0, LPA_MEM_HOST = 1 }; /* where lpa_frame.raw points               */

/* Sample storage between raw decode and the fit:
 *   FUSED   raw samples are decoded straight into LDS by the fit kernel;
 *   FP32    a pre-pass writes FP32 radiance + FP32 inverse variance planes;
 *   FP16    a pre-pass writes the FP16 normalised value (y - o) * 2^-bit_depth,
 *           round-to-nearest-even, +Inf for masked samples (masking is
 *           decided on the raw value); the fit kernel decodes radiance and
 *           variance from it.  For ADCs of up to 12 bits o = 2^(bit_depth-1):
 *           FP16 holds every integer in [-2048, 2048] exactly, so the raw
 *           values are stored without loss and the results equal FUSED's bit
 *           for bit.  Deeper ADCs use o = black_level: values up to 2048 DN
 *           above it are exact, larger ones carry 2^-12 relative rounding. */
enum { LPA_STORE_FUSED = 0, LPA_STORE_FP32 = 1, LPA_STORE_FP16 = 2 };

/* lpa_params.flags */
/* Valid fits keep the values of their FP32 moments: no FP64 values for fits
 * whose pivot is below tau_fp64 nor for the value_tol target.  Fits whose
 * validity the FP32 pivots cannot decide are still decided (and then valued)
 * on FP64 moments. */
#define LPA_FLAG_NO_FP64_FALLBACK 0x1u
/* Pre-computed window weights (Sec. 8: the paper precomputes the weights for
 * registered sensors at the output resolution).  When every sensor map T_s
 * and the output map O are translations (linear parts exactly the identity),
 * the in-window samples of an output pixel, their window weights and their
 * monomials depend only on the pixel's 2x2 parity; the rig tabulates them
 * once per parameter class (radii, windows, output translation) in device
 * memory charged to the context's budget and kept until lpa_destroy_rig.  The
 * first call of a class builds and uploads its table (blocking).  Same
 * estimator, validity and ICI rules as the general path; the results agree
 * with it to rounding (the weights are computed in FP64 and rounded once),
 * not bit for bit.  Per-frame calls only (lpa_reconstruct,
 * lpa_reconstruct_plain), isotropic windows only (mode LPA), 16x16 tiles.
 * Errors: LPA_ERR_UNSUPPORTED for rigs or output maps that are not
 * translations, CALPA, batches, lpa_submit and lpa_autotune;
 * LPA_ERR_OOM if the table exceeds the budget. */
#define LPA_FLAG_PRECOMPUTED_WEIGHTS 0x2u

/* Optional per-pixel calibration frames of one sensor (Sec. 6: the bias frame
 * b_i, the photo-response non-uniformity a_i, the readout variance Var[r_i]
 * and the saturation frame; plus a defect mask).  Host memory, width * height
 * values each, row-major with no padding; copied to the device by
 * lpa_create_rig (the caller may free them afterwards).  A NULL frame selects
 * the sensor's scalar (black_level, a = 1, read_sigma^2, saturation; no
 * defects).  With frames, a sample at pixel i is
 *   f = (y - b_i) / (g n a_i),  Var f = (g max(y - b_i, 0) + Var[r_i]) / (g n a_i)^2,
 * and it is masked iff y >= saturation_i or defect_i != 0.  Validation (at
 * lpa_create_rig, LPA_ERR_INVALID_ARG): every b_i finite, a_i > 0 and finite,
 * Var[r_i] > 0 and finite with the FP32 inverse variance of a dark sample in
 * range, saturation_i not NaN.  Device memory: 16 bytes per pixel of a sensor
 * that has any frame, charged to the context's budget until lpa_destroy_rig. */
typedef struct {
  const float* bias;       /* b_i [DN]                  */
  const float* prnu;       /* a_i (> 0)                 */
  const float* read_var;   /* Var[r_i] [DN^2] (> 0)     */
  const float* saturation; /* masked iff y >= this [DN] */
  const uint8_t* defect;   /* nonzero: never used       */
} lpa_calib;

/* One sensor of a rig (Sec. 3, Sec. 4, Sec. 6). */
typedef struct {
  int32_t width, height; /* pixels                                          */
  int32_t cfa;           /* LPA_CFA_*                                       */
  int32_t bit_depth;     /* ADC bits (FP16 storage normalises by 2^bits)    */
  double affine[6];      /* T_s: sensor pixel centre -> reference plane     */
  double exposure;       /* n_s * t_s (relative exposure, > 0)              */
  double gain;           /* g_s [DN / e-] (> 0)                             */
  double read_sigma;     /* sqrt(Var[r_s]) [DN] (> 0)                       */
  double black_level;    /* b_s [DN]                                        */
  double saturation;     /* a sample is masked iff y >= saturation [DN]     */
  const lpa_calib* calib;/* optional per-pixel frames (NULL: scalars only)  */
} lpa_sensor_desc;

typedef struct {
  int32_t n_sensors; /* 1..LPA_MAX_SENSORS */
  const lpa_sensor_desc* sensors;
} lpa_rig_desc;

/* Reconstruction parameters (Sec. 5.3: order M, window, scale). */
typedef struct {
  int32_t out_w, out_h;   /* output grid                                            */
  double out_affine[6];   /* O: output pixel (u = col, v = row) -> reference plane  */
  int32_t order;          /* M in {0, 1, 2}                                         */
  int32_t n_scales;       /* 1..LPA_MAX_SCALES window radii                         */
  double radii[LPA_MAX_SCALES]; /* ascending, > 0                                   */
  double h[LPA_MAX_SCALES];     /* window parameter; <= 0 selects 2 r^2 / 9         */
  double gamma;           /* ICI interval half-width in standard deviations (> 0)  */
  double green_ratio;     /* green radius / h scale kappa_G (> 0; 1 = same as R/B)  */
  int32_t storage;        /* LPA_STORE_*                                            */
  double tau_inv;         /* validity threshold; <= 0 selects 1e-5                  */
  double tau_fp64;        /* order-2 solves with a smaller pivot are refined in FP64 (<= 0: 1e-3) */
  uint32_t flags;         /* LPA_FLAG_*                                             */
  /* Adaptive anisotropic LPA with colour-channel correlation (CALPA, Sec. 5.4 and
   * 5.5), used when mode == LPA_MODE_CALPA:
   *   1. the gradient of an isotropic fit of the G channel (radius grad_radius,
   *      scaled by green_ratio like every G window; order grad_order) at every
   *      output pixel;
   *   2. per output pixel, the singular values s1 >= s2 and directions of the
   *      gradients of the (2 grad_halfwin + 1)^2 surrounding output pixels
   *      give the steering matrix C = gamma U diag(sigma, 1/sigma) U^T, with
   *      sigma = (s1 + lambda1) / (s2 + lambda1) across the edge,
   *      gamma = ((s1 s2 + lambda2) / M)^alpha, M the pixels counted; both
   *      eigenvalues are clamped to [1/max_stretch^2, max_stretch^2];
   *   3. the order-M ICI reconstruction of R, G and B with the window
   *      exp(-d^T C d / h) - exp(-r^2 / h) on the ellipse d^T C d < r^2.
   * Zero values select: grad_radius the second radius (the first if there is
   * one), grad_h 2 r^2 / 9, max_stretch 2, grad_order 1.  lambda1, lambda2
   * are in the units of the squared gradient (radiance per reference pixel);
   * the paper uses 1 and 0.001.  CALPA frames are reconstructed per frame
   * (lpa_reconstruct, lpa_reconstruct_plain); batches and lpa_submit reject
   * them with LPA_ERR_UNSUPPORTED. */
  int32_t mode;           /* LPA_MODE_*                                             */
  int32_t grad_order;     /* 1 or 2 (0: 1)                                          */
  int32_t grad_halfwin;   /* >= 0                                                   */
  int32_t pad_;
  double alpha;           /* structure sensitivity >= 0                             */
  double lambda1, lambda2;/* lambda1 > 0 (flat windows: s1 = s2 = 0), lambda2 >= 0   */
  double grad_radius;     /* reference-plane units (<= 0: default)                  */
  double grad_h;          /* <= 0: 2 grad_radius^2 / 9                              */
  double max_stretch;     /* >= 1 (0: 2)                                            */
  /* Accuracy target of the output values, relative to max(|C0|, floor) with
   * floor = 1 / max_s(g_s n_s) (one DN of the most exposed sensor).  Moments
   * are accumulated in FP32; with every fit the kernel computes a bound S on
   * how far the rounding of its moment terms can move C0 (per unit relative
   * rounding; an upper estimate of the componentwise condition of C0 in the
   * moment terms, plus a term for window weights computed from FP32 offsets),
   * and where 8 * 2^-24 * S exceeds value_tol times the scale above, the
   * chosen fit of that output is recomputed in FP64 from the raw frame (the
   * decode, the sample positions, the window and the sums all in FP64).  In
   * HDR windows C0 is often a small difference of large terms, so a few
   * percent of the outputs of the benchmark frame take this path.  0 selects
   * 1e-4; a negative value never recomputes. */
  double value_tol;
  /* Temporal scale per radius, in frames^2 (lpa_reconstruct_temporal only):
   * a sample of the frame at time -t has its window multiplied by
   * exp(-t^2 / h_t[m]) at radius m; 0 keeps only the output's frame.  Else
   * at least (n_times - 1)^2 / 16 (the oldest frame's factor >= e^-16). */
  double h_t[LPA_MAX_SCALES];
} lpa_params;

enum { LPA_MODE_LPA = 0, LPA_MODE_CALPA = 1 };

/* One frame: a raw plane per sensor (row-major, row_pitch_bytes apart). */
typedef struct {
  int32_t n_sensors;
  const void* raw[LPA_MAX_SENSORS];
  int64_t row_pitch_bytes[LPA_MAX_SENSORS];
  int32_t dtype;  /* LPA_DTYPE_*                                   */
  int32_t memory; /* LPA_MEM_*: lpa_reconstruct needs DEVICE;       */
                  /* lpa_submit accepts HOST (copied at admission)  */
} lpa_frame;

/* Output: RGB float32, pixel-interleaved rows; optional per-channel code map
 * (order_used << 4 | radius index, 0xFF where nothing is valid) and optional
 * per-channel standard deviation of the output value (the square root of the
 * estimator's variance, NaN where nothing is valid).  Device pointers. */
typedef struct {
  float* rgb;
  int64_t row_pitch_bytes;
  uint8_t* scale_map;         /* may be NULL                     */
  int64_t scale_map_pitch;    /* bytes between scale_map rows    */
  float* sd_map;              /* may be NULL                     */
  int64_t sd_map_pitch;       /* bytes between sd_map rows       */
  /* CALPA only, both optional: the G gradient of every output pixel (2 floats,
   * reference-plane units, zero where its fit is invalid) and the steering
   * matrix (4 floats: cxx, cxy, cyy, 0). */
  float* grad_map;
  int64_t grad_map_pitch;
  float* steer_map;
  int64_t steer_map_pitch;
  /* Optional device pointer to two counters, written stream-ordered after the
   * frame: [0] outputs (pixel x channel) whose value came from an FP64 solve,
   * [1] outputs with no valid fit (NaN).  lpa_submit also reports them in
   * lpa_result. */
  uint64_t* stats;
} lpa_output;

/* Status and timestamps of a submitted frame (CLOCK_MONOTONIC ns). */
typedef struct {
  int32_t status;         /* LPA_OK, LPA_NOT_READY or an error */
  int32_t batch_size;     /* frames in the launch that ran it  */
  int64_t t_arrival_ns, t_admit_ns, t_start_ns, t_done_ns;
  uint64_t n_fp64;        /* outputs valued by an FP64 solve (as lpa_output.stats[0]) */
  uint64_t n_invalid;     /* outputs with no valid fit (NaN) */
} lpa_result;

typedef struct lpa_ctx lpa_ctx;
typedef struct lpa_rig lpa_rig;

/* Create a context on HIP device `device` with an HBM budget (bytes) for the
 * library's own buffers (0 = 90% of free memory).  The context owns its
 * streams, scratch planes, autotune cache and serving scheduler. */
lpa_status lpa_create_ctx(int device, size_t hbm_budget_bytes, lpa_ctx** out);
/* Wait for all work of the context, stop its scheduler, free everything,
 * including rigs not yet destroyed (their handles become invalid). */
lpa_status lpa_destroy_ctx(lpa_ctx* ctx);

/* Create a rig: the descriptor is validated and copied (caller may free it);
 * the per-sensor calibration and noise constants stay resident on the
 * device until lpa_destroy_rig.  Validation: 1..8 sensors, sizes >= 1,
 * gain, exposure, read_sigma > 0, invertible affine, finite values,
 * saturation > black_level, 1 <= bit_depth <= 16. */
lpa_status lpa_create_rig(lpa_ctx* ctx, const lpa_rig_desc* desc, lpa_rig** out);
/* Waits for the context's queued and running work, then frees the rig. */
lpa_status lpa_destroy_rig(lpa_rig* rig);

/* Reconstruct one frame, stream-ordered on `hip_stream` (a hipStream_t; NULL
 * = the null stream).  raw and out are device pointers borrowed until the
 * stream passes this work.  Returns after enqueueing.  When wide windows over
 * many sensors make a tile's staged samples overflow the workgroup's 64 KiB
 * of LDS, the launch uses smaller tiles (down to 4x4 output pixels); a window
 * no tile can stage, or one more than 240 sensor pixels across, returns
 * LPA_ERR_UNSUPPORTED before anything is enqueued. */
lpa_status lpa_reconstruct(lpa_rig* rig, const lpa_frame* frame, const lpa_params* params,
                           const lpa_output* out, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * reconstruction as lpa_reconstruct (same kernels, same tuned launch shape,
 * bit-identical results) for mode LPA with storage FUSED, with every scratch
 * buffer in a static 16 MiB device array per GPU instead of the context's
 * stream-ordered allocations.  It calls no hipMalloc / hipFree.  The array
 * holds the refit marks (3 bytes per output pixel) and, if out->stats is set,
 * the per-tile counts (8 bytes per tile): outputs beyond about 5.5 Mpixel
 * return LPA_ERR_UNSUPPORTED, as do CALPA, the pre-pass storage forms and
 * LPA_FLAG_PRECOMPUTED_WEIGHTS.  Every call on one GPU shares its array:
 * calls that overlap on one GPU (other streams, other threads) race and must
 * be serialised by the caller. */
lpa_status lpa_reconstruct_noalloc(lpa_rig* rig, const lpa_frame* frame, const lpa_params* params,
                                   const lpa_output* out, void* hip_stream);

/* The plain per-frame form: FP32 radiance / inverse-variance planes from a
 * separate pre-pass launch, then one fit launch with 16x16 tiles (no tuning;
 * smaller tiles only where the LDS rule above requires them).  Same results
 * contract as lpa_reconstruct. */
lpa_status lpa_reconstruct_plain(lpa_rig* rig, const lpa_frame* frame, const lpa_params* params,
                                 const lpa_output* out, void* hip_stream);

/* Reconstruct n frames (each with its own rig and parameters) in one
 * persistent launch that pulls output tiles from a device work queue.  The
 * launch is recorded into a HIP graph and replayed while the frame shapes
 * are unchanged (`reuse` != 0 lets the library keep that graph).  Each
 * frame's result is bit-identical to lpa_reconstruct of that frame alone. */
lpa_status lpa_reconstruct_batch(lpa_ctx* ctx, int32_t n, lpa_rig* const* rigs,
                                 const lpa_frame* frames, const lpa_params* params,
                                 const lpa_output* outs, void* hip_stream);

/* Serving: queue a frame that arrived at `arrival_ns` (CLOCK_MONOTONIC).  Host
 * raw planes are copied into a device slot when the HBM budget admits the
 * frame; frames admitted while others run are batched into the next launch,
 * which overlaps the running one on a second stream.  raw and out are
 * borrowed until lpa_poll reports a terminal status.  The library's copies
 * and launches run on its own non-blocking streams, unordered with the
 * caller's: work the caller enqueued on raw or out must be complete before
 * the call.  Returns LPA_AGAIN if the admission queue (1024 frames) is full. */
/* A frame none of the batch tile shapes (16x16, 32x8, 8x32, 64x4 output
 * pixels) can stage is refused here with LPA_ERR_UNSUPPORTED; a frame that
 * cannot fit the HBM budget beside what the context holds while no served
 * frame is in flight finishes with LPA_ERR_OOM. */
lpa_status lpa_submit(lpa_rig* rig, const lpa_frame* frame, const lpa_params* params,
                      const lpa_output* out, int64_t arrival_ns, uint64_t* ticket);
/* Non-blocking: LPA_NOT_READY until the frame is done; then its result,
 * handed out once: the ticket is forgotten after that (a later poll returns
 * LPA_ERR_INVALID_ARG), so the context keeps no record of collected frames. */
lpa_status lpa_poll(lpa_ctx* ctx, uint64_t ticket, lpa_result* out);
/* Block until every submitted frame is finished.  After a device error the
 * context is failed: frames not yet launched finish with LPA_ERR_DEVICE,
 * submissions are refused, and the context is to be destroyed (a new one
 * can be created on the device).  For tests, the environment variable
 * LPA_TEST_FAIL_AFTER=N, read when a context is created, makes its N-th
 * serving batch launch fail this way from the host, before any GPU work. */
lpa_status lpa_drain(lpa_ctx* ctx);

/* Autotuning (launch shape only; results never depend on it).  Candidates:
 * tile shapes 16x16, 32x8, 8x32, 64x4 output pixels (256 lanes; a wavefront
 * holds one 2x2 parity class of the tile: 8x8, 16x4, 4x16 or 32x2 pixels two
 * apart) times two register budgets for
 * order-2 fits (3 or 4 waves per SIMD).  Each candidate is launched on the
 * given frame `reps` times on `hip_stream` (writing `out`), timed with HIP
 * events; the fastest becomes the choice for every frame of the same class
 * (order, radii, sensor count, storage, output zoom) in this context.
 * Blocks until the timing is done. */
typedef struct {
  int32_t tile_w, tile_h, occupancy, n_candidates;
  double ms_best, ms_default; /* per launch; default = 16x16, default registers */
} lpa_tune_result;
lpa_status lpa_autotune(lpa_rig* rig, const lpa_frame* frame, const lpa_params* params,
                        const lpa_output* out, void* hip_stream, int32_t reps, lpa_tune_result* result);
/* Persist / restore the context's tuning choices (small JSON file). */
lpa_status lpa_tuner_save(lpa_ctx* ctx, const char* path);
lpa_status lpa_tuner_load(lpa_ctx* ctx, const char* path);

/* Temporal LPA (Sec. 9 names the extension of the supports from space to
 * space and time as future work; this form is a reading of it): frames[t]
 * (t = 0 .. n_times - 1) is the rig's capture at time -t, frames[0] the frame
 * reconstructed.  Every sample's window is the spatial one times
 * exp(-t^2 / params->h_t[m]) for radius m, so ICI selects a spatio-temporal
 * scale and shrinks the support where the frames disagree (no motion
 * compensation); the local model is constant in t.  Mode LPA, isotropic
 * windows, storage FUSED (raw frames read by the fit kernel), device frames
 * of one dtype; n_times * n_sensors <= LPA_MAX_SENSORS (the kernel stages
 * each frame's sensors as sensors of their own).  Outputs, validation and
 * errors as lpa_reconstruct; LPA_ERR_UNSUPPORTED for other modes, storage
 * forms and flags. */
lpa_status lpa_reconstruct_temporal(lpa_rig* rig, const lpa_frame* frames, int32_t n_times,
                                    const lpa_params* params, const lpa_output* out, void* hip_stream);

/* Kernel timing, a profiling aid.  While it is on, every lpa_reconstruct and
 * lpa_reconstruct_plain on the context (not the allocation-free form) brackets
 * its fit launch (isotropic, pre-computed-weight or, for CALPA, steered) and
 * its FP64 refit launch with HIP events on the caller's stream.
 * lpa_kernel_times waits for every bracketed launch recorded since timing was
 * switched on or last read, returns the total milliseconds and launch counts
 * of each kernel, and clears the records.  Switching it on or off clears
 * them too.  Off by default: then no event is recorded.  The brackets include
 * the gaps between back-to-back launches (a few microseconds). */
typedef struct {
  double fit_ms, refit_ms;     /* summed launch durations */
  int64_t n_fit, n_refit;      /* bracketed launches */
} lpa_kernel_time;
lpa_status lpa_set_kernel_timing(lpa_ctx* ctx, int32_t on);
lpa_status lpa_kernel_times(lpa_ctx* ctx, lpa_kernel_time* out);

/* Thread-local message of the last non-OK status returned on this thread. */
const char* lpa_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
