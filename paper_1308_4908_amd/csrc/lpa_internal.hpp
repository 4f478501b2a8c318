// lpa_internal.hpp -- launch descriptors shared by the host library and the
// gfx950 kernels.  Everything a fit launch needs is precomputed on the host in
// FP64 and packed here; the kernels read it through scalar loads.
#pragma once

#include <stdint.h>

#include <hip/hip_runtime.h>

namespace lpa {

constexpr int kMaxSensors = 8;
constexpr int kMaxScales = 8;

// Where the fit kernel reads samples from.
enum SrcKind : int32_t {
  SRC_RAW_U16 = 0,   // raw uint16 DN, decoded while staging (fused)
  SRC_RAW_F32 = 1,   // raw float DN (test input), decoded while staging (fused)
  SRC_PLANE_F32 = 2, // float2 (radiance, inverse variance) plane from a pre-pass
  SRC_PLANE_F16 = 3, // half normalised radiance plane from a pre-pass (+Inf = masked)
};

// Per-sensor constants of one launch.
struct SensorK {
  double fwd[6];        // T_s: X = f0 x + f1 y + f2, Y = f3 x + f4 y + f5
  double inv[6];        // T_s^-1
  double wmax[2];       // largest box half-width (sensor px) along x, y over all scales/channels
  double rownorm[2];    // |row 0|, |row 1| of the inverse linear part
  const void* src;      // raw plane or pre-pass plane (device)
  int64_t pitch;        // bytes between rows of src
  float inv_ge;         // 1 / (g n)
  float gain;           // g
  float read_var;       // sigma_r^2 [DN^2]
  float black;          // b [DN]
  float sat;            // saturation [DN]
  float norm_decode;    // 2^bit_depth: FP16 plane value v -> y = v 2^bits + norm_offset
  float norm_offset;    // 2^(bit_depth - 1) up to 12 bits (lossless), else the black level
  int32_t width, height;
  int32_t reg_w, reg_h; // LDS region bound (samples) for the launch's tile shape
  int32_t lds_off;      // region offset in the LDS sample array (float2 units)
  int8_t sub_n[3];      // number of CFA sub-lattices of channel c (1 or 2)
  int8_t sub_ox[3][2];  // sub-lattice column parity
  int8_t sub_oy[3][2];  // sub-lattice row parity
  int8_t nbox[2][kMaxScales][2]; // box size (sub-lattice points) [class][scale][x|y]
  int8_t pad_[5];
  // per-pixel calibration (row-major width*height), or null for the scalars:
  // (b_i, a_i, Var[r_i], saturation_i), saturation -inf for defects
  const float4* calib;
  // The frame's raw plane (also for the pre-pass forms) and the noise model in
  // FP64, read by the FP64 refit of outputs whose FP32 value is not accurate
  // enough.
  const void* raw;
  int64_t raw_pitch;    // bytes
  int32_t raw_f32;      // raw samples are float DN (else uint16)
  int32_t time;         // temporal LPA: the frame's time is -time (0: the output's frame)
  double gain64, ge64, inv_ge64;  // g, g n, 1 / (g n)
  double black64, read_var64, sat64;
  float kt[kMaxScales]; // temporal LPA: exp(-time^2 / h_t) per radius (1 at time 0, 0 for h_t = 0)
};

// Per-scale constants, per channel class (0: R and B, 1: G).
struct ScaleK {
  double radius[2];   // r' = r * kappa_class
  double box_radius[2]; // half-width of the support box: r', or r' times the stretch bound of steered windows
  float coord_scale[2]; // s = sqrt(log2(e) / h'): exp(-|d|^2 / h') = exp2(-|s d|^2)
  float reach2[2];    // (s r' (1 + 1e-4))^2: samples at or beyond it have exactly zero weight
  float e_edge[2];    // exp(-r'^2 / h'): subtracted so the window vanishes at r'
  double h[2];        // h' = h * kappa_class^2 (FP64 refit)
  // Rounding bound of window weights from FP32 offsets: an offset's rounding
  // moves |s d|^2 by up to a few u |s d|^2, the weight by ln2 2^-|s d|^2 times
  // that, which the moment bound covers except for a part up to
  // ln2 e_edge R^2 (R = s r') times iv per sample; edge_coef is that factor
  // (with the offsets' rounding multiple, over the moment bound's), mono_r
  // bounds |s dx|, |s dy| on the isotropic window (s r', a steered window
  // scales it by its own extent).
  float edge_coef[2];
  float mono_r[2];
  double inv_ht;      // temporal LPA: 1 / h_t (frames^-2) of this radius
};

// Pre-computed window weights (rigs whose sensor maps and output map are
// translations, Sec. 8): the offset from an output pixel to the channel-c
// samples of a sensor depends only on the pixel's 2x2 parity, so the window
// weight K and the scaled monomials of every in-window sample are fixed per
// (channel, parity, radius index, sensor) and tabulated once.
struct StencilEntry {
  float a[15];      // K * monomial (Hankel order: 1, x, y, x^2, xy, y^2, x^3, x^2y, xy^2, y^3, x^4, ..., y^4),
                    // scaled offsets; a[0] is the window weight K
  int32_t delta;    // LDS offset of the sample from output pixel (u, v)'s own position, l * reg_w + k for
                    // sample = (u + k, v + l) in sensor pixels (tiles staged with row pitch reg_w)
};
static_assert(sizeof(StencilEntry) == 64, "stencil entry layout: one 64-byte scalar load");

struct StencilSeg {
  int32_t off, n;   // first entry and entry count
};

// Device table: the segment index followed by the entries.
struct StencilTable {
  StencilSeg seg[3][4][kMaxScales][kMaxSensors];  // [channel][parity: (u & 1) + 2 (v & 1)][radius][sensor]
  // StencilEntry entries[] follow at entries_offset()
  static constexpr size_t entries_offset() { return (sizeof(StencilSeg) * 3 * 4 * kMaxScales * kMaxSensors + 255) / 256 * 256; }
};

struct LaunchK {
  double out_affine[6];
  int32_t out_w, out_h;
  int32_t tiles_x, tiles_y; // tile grid of this frame
  int32_t tile_w, tile_h;
  int32_t n_sensors, n_scales;
  int32_t order, src_kind;
  float gamma, tau_inv, tau_fp64;
  int32_t use_fp64;
  int32_t lds_floats2;      // float2 elements of LDS this launch uses
  int32_t need_var;         // estimator variance needed (several radii or an sd map)
  int32_t occupancy;        // 0: default register budget; 4: compiled for 4 waves/SIMD (order 2)
  // Output values are recomputed from FP64 moments where the FP32 moments'
  // rounding could move them by more than the target: when the bound S on
  // |dC0| per unit relative rounding of the moment terms exceeds
  // risk_max * max(|C0|, value_floor) (risk_max = +inf: never).
  float risk_max;
  float value_floor;        // one DN of the most exposed sensor, in radiance units
  int32_t refit_lds;
  // optional per-tile counts (2 x uint32 per tile: outputs whose value came
  // from an FP64 solve, outputs with no valid fit), indexed by the frame's
  // tile number; null: not counted
  uint32_t* tile_stats;
  uint64_t* frame_stats;    // where the batch's count reduction writes this frame's sums (or null)
  // per output (pixel x channel) byte: 0x80 | order << 4 | radius index where
  // the output is to be refitted in FP64, else 0; written by the fit, read by
  // the refit launch (null: no refit)
  uint8_t* refit_map;
  int64_t refit_pitch;      // bytes
  // FP64 refit blocks: refit_bw x refit_bh output pixels per workgroup (at
  // most 32 x 32), staging refit_lds raw DN (the sensors' block footprints)
  int32_t refit_bw, refit_bh;
  float* rgb;
  int64_t rgb_pitch;        // bytes
  uint8_t* map;
  int64_t map_pitch;        // bytes
  float* sd;                // optional standard deviation of each output value
  int64_t sd_pitch;         // bytes
  const float* steer;       // steered fit: per output pixel (cxx, cxy, cyy, 0) of the window d^T C d
  int64_t steer_pitch;      // bytes
  float* grad;              // gradient pass: per output pixel (df/dX, df/dY), reference-plane units
  int64_t grad_pitch;       // bytes
  const StencilTable* stencil; // pre-computed-weight fit: the launch's table (device)
  SensorK s[kMaxSensors];
  ScaleK sc[kMaxScales];
};

// Output pixel offset (du, dv) of thread tid within a tw x th tile (both even).
// The threads are split into the four 2x2 parity classes of output pixels,
// each laid out row-major over the tile's pixels of that parity, so a 64-lane
// wave holds pixels two apart: their positions relative to a sensor's CFA
// lattice differ only by the slow drift of the rig's rotation and scale, and
// a sample outside one lane's window is then mostly outside all of them.
#if defined(__HIPCC__)
__host__ __device__
#endif
inline void lane_pixel(int tid, int tw, int th, int* du, int* dv) {
  const int per = (tw * th) >> 2;
  const int cls = tid / per, w = tid - cls * per;
  const int hw = tw >> 1;
  *du = 2 * (w % hw) + (cls & 1);
  *dv = 2 * (w / hw) + (cls >> 1);
}

// Steering pass (adaptive anisotropic windows): per output pixel, the
// structure of the gradients of the (2q+1)^2 surrounding pixels.
struct SteerArgs {
  const float* grad;        // (df/dX, df/dY) per output pixel
  int64_t grad_pitch;       // bytes
  float* steer;             // (cxx, cxy, cyy, 0) per output pixel
  int64_t steer_pitch;      // bytes
  int32_t out_w, out_h, q, pad_;
  double alpha, lambda1, lambda2;
  double lo, hi;            // eigenvalue clamp [1/kappa^2, kappa^2]
};

// Header of a batch table in device memory (read by the persistent kernel, so
// a captured graph can be replayed with new table contents).
struct BatchHeader {
  int32_t n_frames;
  int32_t pad_;
  int64_t total_tiles;
};

}  // namespace lpa

// Launchers implemented in lpa_kernels.hip (host-callable).
extern "C" {
// Pre-pass over one sensor: raw -> FP32 (radiance, inverse variance) plane or
// FP16 normalised radiance plane.
int lpa_k_prepass(const lpa::SensorK* s, int raw_is_f32, const void* raw, int64_t raw_pitch,
                  void* plane, int64_t plane_pitch, int to_f16, float norm_encode, void* stream);
// One fit launch over the whole tile grid of a frame.
int lpa_k_fit(const lpa::LaunchK* k, void* stream);
// One persistent launch over many frames.
// All frames of one batch share src_kind; each frame's descriptor carries its tile shape
// (block = tile_w * tile_h threads must be the same for all frames).
int lpa_k_fit_batch(const lpa::BatchHeader* d_hdr, const lpa::LaunchK* d_frames,
                    const int64_t* d_first_tile, int32_t* d_queue, int32_t src_kind, int32_t block,
                    int32_t lds_floats2, int32_t grid, void* stream);
int lpa_k_fit_max_lds_bytes(void);
// Gradient pass: K.order (1 or 2) fit of the G channel at radius K.sc[0] (no
// ICI) writing K.grad.
int lpa_k_grad(const lpa::LaunchK* k, void* stream);
// Steering pass over the gradient plane.
int lpa_k_steer(const lpa::SteerArgs* a, void* stream);
// Temporal LPA: the launch's sensors are (frame, sensor) pairs whose kt and
// time are set; raw sources only.
int lpa_k_fit_temporal(const lpa::LaunchK* k, void* stream);
// Fit with pre-computed window weights read from K.stencil (256-lane tiles).
int lpa_k_fit_stencil(const lpa::LaunchK* k, void* stream);
// Fit with per-pixel steered windows read from K.steer.
int lpa_k_fit_steered(const lpa::LaunchK* k, void* stream);
// FP64 refit of the outputs a fit launch marked in K.refit_map (one launch
// over the frame's refit blocks, after the fit on the same stream).
int lpa_k_refit(const lpa::LaunchK* k, void* stream);
// The same for a batch table (after the persistent fit; grid workgroups loop
// over the batch's refit blocks; lds_bytes covers every frame's refit_lds).
int lpa_k_refit_batch(const lpa::BatchHeader* hdr, const lpa::LaunchK* frames, const int64_t* first_tile,
                      int32_t grid, int32_t lds_bytes, int32_t raw_f32, void* stream);
// The graph of one batch, built node by node: copy of the table (copy_bytes
// from pinned h_table to d_table, which holds d_hdr / d_frames / d_first),
// queue reset, persistent fit (grid x block, lds_floats2 float2 of LDS), FP64
// refit (refit_grid workgroups) and count reduction (cap workgroups).
// The fit and refit nodes are returned so that a launch whose frames need
// another LDS size can update them in the instantiated graph
// (lpa_k_batch_graph_set_lds) instead of building a new one.
int lpa_k_batch_graph(hipGraph_t* out, hipGraphNode_t* fit_node, hipGraphNode_t* refit_node, void* d_table,
                      const void* h_table, size_t copy_bytes, const lpa::BatchHeader* d_hdr,
                      const lpa::LaunchK* d_frames, const int64_t* d_first, int32_t* d_queue, int32_t src_kind,
                      int32_t block, int32_t lds_floats2, int32_t refit_lds_bytes, int32_t grid, int32_t refit_grid,
                      int32_t cap, int32_t raw_f32);
int lpa_k_batch_graph_set_lds(hipGraphExec_t exec, hipGraphNode_t fit_node, hipGraphNode_t refit_node,
                              const lpa::BatchHeader* d_hdr, const lpa::LaunchK* d_frames, const int64_t* d_first,
                              int32_t* d_queue, int32_t src_kind, int32_t block, int32_t lds_floats2,
                              int32_t refit_lds_bytes, int32_t grid, int32_t refit_grid, int32_t raw_f32);
// Dynamic LDS a refit launch may take (bytes).
int lpa_k_refit_max_lds_bytes(void);
// Zero n ints with a small kernel (graph-safe replacement for a memset).
int lpa_k_zero_i32(int32_t* p, int32_t n, void* stream);
// Sum a frame's per-tile counts (n_tiles pairs) into out[0], out[1].
int lpa_k_stats_sum(const uint32_t* tile_stats, int64_t n_tiles, uint64_t* out, void* stream);
// The same for every frame of a batch table: workgroup f handles frame f
// (f < hdr->n_frames) if its descriptor carries tile_stats and frame_stats.
int lpa_k_stats_frames(const lpa::BatchHeader* hdr, const lpa::LaunchK* frames, int32_t grid, void* stream);
}
