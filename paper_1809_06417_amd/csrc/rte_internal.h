// Internal declarations shared by the translation units of librte.
// Not part of the public ABI (include/rte.h is).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "rte.h"

namespace rte {

// One wave64 marches one 8x8 pixel tile: a pixel tile is the unit of the
// per-sample weight buffer ("g buffer"), laid out [tile][k / 4][lane][k % 4]:
// four consecutive samples of one ray sit in one 16-byte group, so that the
// 64 rays of a wave write one contiguous 1 KB row every four march steps and
// the back-projection fetches the samples a ray leaves in one voxel (one to
// three at half-voxel steps) with one load. A tile holds kmax rounded up to a
// multiple of kGroup rows.
constexpr int kTile = 8;
constexpr int kTileRays = kTile * kTile;
constexpr int kGroup = 4;

// The back-projection works on bricks of 8 x 8 x 4 cells and sums each
// brick's corner contributions into the brick's 9 x 9 x 5 key points before
// storing them: one plane of kBrickNodeStride floats (405 key points, padded
// to a 128-byte multiple) per accumulator and brick.
constexpr int kBrickNodesX = 9, kBrickNodesY = 9, kBrickNodesZ = 5;
constexpr int kBrickNodes = kBrickNodesX * kBrickNodesY * kBrickNodesZ;
constexpr int kBrickNodeStride = 416;

// Plan-free render (rte_render_static): its workspaces live in one static
// device array of kStaticScratchBytes per GPU; at most kStaticMaxViews
// cameras, which travel in the kernel arguments.
constexpr size_t kStaticScratchBytes = RTE_STATIC_SCRATCH_BYTES;
constexpr int kStaticMaxViews = RTE_STATIC_MAX_VIEWS;

// Back-projection / epilogue selectors shared by launch wrappers and kernels.
enum ResidualMode : int {
    kEpiImage = 0,  // write I_c
    kEpiSart = 1,   // y_c = (F_c - I_c) / R, R = sum_k g_k (0 where R = 0)
    kEpiMlem = 2,   // y_c = F_c / I_c (1 where I_c <= 0)
    kEpiPaper = 3,  // y_c = F_c - I_c
};

enum GatherMode : int {
    kGatherAdjoint = 0,       // acc_c += g * y_c * w
    kGatherAdjointCols = 1,   // acc_c += g * y_c * w ; acc_C += g * w
    kGatherPaper = 3,         // acc_c += alpha_l y_c (1-tau)^k exp(-alpha_d D)
    kGatherGrad = 4,          // acc_c += g * y_c * w ; acc_C += q * w
    kGatherHull = 5,          // bit v set when a flame ray of view v has a sample in the cell
};

enum UpdateMode : int {
    kUpdDelta = 0,   // out[c][j] = sum
    kUpdSart = 2,    // e += lambda sum / cols (cols > 0)
    kUpdMlem = 3,    // e *= 1 + lambda (sum / cols - 1) (cols > 0)
    kUpdPaper = 4,   // e += sum
    kUpdTemp = 5,    // EM on the fitted channel, clamp to LUT, invert to T
    kUpdGrad = 6,    // out[c][j] = sum_c, out2[j] = sum_C (emission / extinction gradients)
    kUpdSartOS = 7,  // SART with the column sums gathered alongside (sum_C): ordered subsets and
                     // the first iteration (which also stores them in cols_out)
    kUpdMlemOS = 8,  // EM likewise
};

// Per-view projection from voxel coordinates to homogeneous pixel
// coordinates: (hu, hv, hw) = P[0..3] . (X,1), P[4..7] . (X,1), P[8..11] . (X,1).
struct ViewProj {
    float P[12];
};

struct TimingRecord {
    int kernel;
    hipEvent_t start, stop;
};

}  // namespace rte

struct rte_plan {
    // configuration
    rte_grid grid{};
    rte_render_params params{};
    std::vector<rte_camera> cams;
    int V = 0, W = 0, H = 0;
    int tiles_x = 0, tiles_y = 0, tiles_per_view = 0, n_tiles = 0;
    int64_t n_rays = 0, n_nodes = 0, n_cells = 0;
    int64_t n_part_cells = 0;  // cells rounded up to whole 8x8x4 gather bricks
    double h[3] = {0, 0, 0};
    double ds = 0.0;
    uint64_t samples = 0, hit_rays = 0, g_floats = 0;
    int scat_nup = 0;  // in-scatter directions 0 .. scat_nup-1 point up (z >= 0), the rest down
    hipStream_t last_stream = nullptr;

    // device workspaces (all owned by the plan)
    rte_camera *d_cams = nullptr;
    rte::ViewProj *d_proj = nullptr;
    float4 *d_rayA = nullptr;       // entry point (voxel coords) xyz, chord length w
    float4 *d_rayB = nullptr;       // direction (voxel units per world unit) xyz, K (int bits) w
    float *d_tnear = nullptr;       // entry distance (export only)
    int32_t *d_tile_kmax = nullptr;
    uint32_t *d_tile_off = nullptr;  // per tile: first slot in d_g (plans keep < 2^32 slots)
    int32_t *d_tile_order = nullptr; // launch slots: tiles with samples (per-XCD bands, -1 for an empty slot), then tiles without
    int n_active_slots = 0;         // slots of the tiles with samples
    int n_slots = 0;                // all slots (entries of d_tile_order and of d_err)
    float *d_g = nullptr;           // per-sample weights T_k Delta_k phi_k, [tile][k / 4][lane][k % 4]
    float *d_q = nullptr;           // gradient plans: per-sample (g_k, q_k) float2 pairs, [tile][K - 1 - k][lane] from the d_g tile offsets
    float *d_vol = nullptr;         // packed volume: float4 (C = 3) or float2 (C = 1)
    float4 *d_scat = nullptr;       // packed in-scatter grid (rgb, 0)
    float4 *d_dirs = nullptr;       // in-scatter directions, voxel units per world unit
    double *d_dirs_world = nullptr; // the same directions in the world frame [kMaxDirs][3]
    float *d_scat_part = nullptr;   // per-direction in-scatter sums [dirs][C][M^3]
    float *d_y = nullptr;           // per-pixel residual values [V][C][H][W]
    float *d_part = nullptr;        // per-cell corner partials [8][acc][cells]
    float *d_cols = nullptr;        // column sums A^T 1 [N]
    float *d_lut = nullptr;         // [3][lut_cap]
    float *d_mask = nullptr;        // flame-pixel mask [V][H][W]
    int32_t *d_inside = nullptr;    // visual-hull flag per key point [N]
    float2 *d_err = nullptr;        // per-tile (squared residual, count) of the stop rule
    double *d_err_sum = nullptr;    // reduced (sum, count)
    double *h_err_sum = nullptr;    // pinned host copy
    int last_iters = 0;             // updates made by the last reconstruction
    // open job (rte_job_begin .. rte_job_end)
    bool job_open = false;
    const float *job_frames = nullptr;
    rte_recon_params job_params{};
    int job_iter = 0;
    void *d_batch = nullptr;        // device copy of batched launch arguments
    void *h_batch = nullptr;        // pinned host staging of the same
    hipEvent_t batch_event = nullptr;  // marks the end of the last upload from h_batch
    size_t batch_bytes = 0;            // [0, batch_bytes): render, gather and update arguments
    size_t scat_stage_off = 0, scat_stage_bytes = 0;  // region of batched in-scatter arguments
    hipEvent_t scat_event = nullptr;   // marks the end of the last upload from that region
    std::vector<float> last_errors; // image RMS per iteration of the last reconstruction (stop rule)
    int lut_cap = 0;
    int part_acc = 0;               // accumulators per corner the partial buffer holds
    size_t device_bytes = 0;

    // LUT cache key
    bool lut_valid = false;
    rte_temp_params lut_params{};
    std::vector<float> lut_host;

    // timing
    uint32_t timing_mask = 0;  // bit k: launches of RTE_KERNEL k are bracketed by events
    std::vector<rte::TimingRecord> pending;
    std::vector<hipEvent_t> event_pool;
    double kernel_ms[RTE_KERNEL_COUNT] = {0};
    int64_t kernel_launches[RTE_KERNEL_COUNT] = {0};
};

namespace rte {

// ---- launch wrappers (rte_kernels.hip) ----
hipError_t launch_ray_table(const rte_plan *p, hipStream_t s);
hipError_t launch_tile_kmax(const rte_plan *p, hipStream_t s);
hipError_t launch_ray_export(const rte_plan *p, float *t_near, float *t_far, int32_t *nseg,
                             hipStream_t s);
hipError_t launch_pack(const rte_plan *p, const float *emission, const float *extinction,
                       int channels, hipStream_t s, bool keep_emission = false);
// One iteration of every plan's open job: batched render, gather and update
// launches. marks: NULL or 6 events recorded around the three launches.
hipError_t launch_step_batch(rte_plan *const *plans, int n, hipStream_t s, hipEvent_t *marks = nullptr);
hipError_t launch_unpack(const rte_plan *p, float *emission, int channels, hipStream_t s);
// Residuals in the gather's per-ray layout: packs planar [V][3][H][W] into
// the plan's residual buffer and sets *packed to it (one channel: to planar).
hipError_t launch_pack_residual(const rte_plan *p, const float *planar, const float **packed, hipStream_t s);
hipError_t launch_pack_scatter(const rte_plan *p, const float *planar, hipStream_t s);
hipError_t launch_render(const rte_plan *p, int channels, bool use_emission, bool use_scatter,
                         bool write_g, int epilogue, const float *frames, int frame_channels,
                         int frame_channel0, float *out, hipStream_t s, double *exit_tau = nullptr,
                         const float *mask = nullptr, float2 *err = nullptr, int sub_n = 1, int sub_s = 0);
hipError_t launch_adjoint_march(const rte_plan *p, bool use_scatter, const double *exit_tau, const float *dI,
                                hipStream_t s);
hipError_t launch_inscatter(const rte_plan *p, float *planar_out, hipStream_t s);
// The in-scatter grids of n plans with one launch per march pass and reduce
// (arguments staged through plans[0]'s in-scatter region).
hipError_t launch_inscatter_batch(rte_plan *const *plans, int n, hipStream_t s);
hipError_t launch_gather(const rte_plan *p, int channels, int mode, const float *y,
                         float alpha_l, float alpha_d, float tau, hipStream_t s,
                         const float *rowmask = nullptr, float g_sigma = 0.f, uint64_t seed = 0,
                         int iteration = 0, int view0 = 0, int view_step = 1);
hipError_t launch_flame_mask(const rte_plan *p, const float *frames, int frame_channels, float threshold,
                             float *mask, hipStream_t s);
hipError_t launch_hull(const rte_plan *p, const float *mask, int32_t *inside, hipStream_t s);
hipError_t launch_apply_outside(const rte_plan *p, int channels, const int32_t *inside, float value,
                                hipStream_t s);
hipError_t launch_err_reduce(const rte_plan *p, double *out, hipStream_t s);
hipError_t launch_update(const rte_plan *p, int channels, int acc, int mode, float lambda,
                         int clamp_nonneg, float *out, float *temperature, int lut_size,
                         int fit_channel, hipStream_t s, float *out2 = nullptr,
                         const int32_t *inside = nullptr, float *cols_out = nullptr);
hipError_t launch_temp_map(const rte_plan *p, const float *T, float *em_planar, float *sig_planar,
                           bool packed, int lut_size, int fit_channel, float sigma_max,
                           float soot_t0, float soot_span, float t_min, float t_max,
                           hipStream_t s);
hipError_t launch_temp_invert(const rte_plan *p, const float *e, float *T, int lut_size,
                              int fit_channel, float t_min, float t_max, hipStream_t s);

// ---- plan-free render over the static device array ----
// Byte offsets of its workspaces in the array (each 256-byte aligned).
struct StaticLayout {
    size_t cams, rayA, rayB, tnear, order, vol, scat, total;
};
StaticLayout static_layout(int V, int W, int H, int64_t n_nodes, int C, int M, bool per_view_scatter);
// Address of this device's array (looked up once per device).
hipError_t static_scratch(void **addr);
// Ray table, tile list, packing and image render of `view` (a plan whose
// configuration fields are set and whose workspace pointers this call points
// into the array) on stream s.
hipError_t launch_render_static(rte_plan *view, const rte_camera *cams, const float *emission,
                                const float *extinction, const float *inscatter, float *images, hipStream_t s);

// ---- host LUT builder (rte_lut.cpp) ----
void build_temperature_lut(const rte_temp_params &tp, std::vector<float> &lut);

}  // namespace rte
