// C ABI of librte: plan construction, argument validation, workspace and
// HBM budget, kernel sequencing on the caller's stream, per-kernel timing.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "rte_internal.h"

namespace {

thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int ok()
{
    g_last_error.clear();
    return RTE_OK;
}

#define RTE_HIP(call)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail(RTE_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_));      \
    } while (0)

constexpr int kMaxLut = 65536;
constexpr int kMaxBatch = 64;          // plans per rte_job_step
constexpr size_t kBatchBytes = 1 << 17; // staging for their launch arguments
constexpr size_t kScatStageBytes = 1 << 15;  // of which the batched in-scatter's region
constexpr int kMaxDirs = 256;

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

// Validate grid / cameras / params; fills the derived sizes of a plan.
int validate_config(const rte_grid *grid, const rte_camera *cams, int32_t ncams,
                    const rte_render_params *params)
{
    if (!grid || !cams || !params) return fail(RTE_ERR_INVALID_ARG, "null grid, cameras or params");
    if (grid->nx < 2 || grid->ny < 2 || grid->nz < 2)
        return fail(RTE_ERR_INVALID_ARG, "grid needs at least 2 key points per axis (got %d %d %d)",
                    grid->nx, grid->ny, grid->nz);
    for (int i = 0; i < 3; ++i)
        if (!std::isfinite(grid->bbox_min[i]) || !std::isfinite(grid->bbox_max[i]) ||
            !(grid->bbox_max[i] > grid->bbox_min[i]))
            return fail(RTE_ERR_INVALID_ARG, "bbox axis %d is empty or not finite", i);
    const int64_t nodes = (int64_t)grid->nx * grid->ny * grid->nz;
    if (nodes >= (int64_t(1) << 27) || (int64_t)grid->nx * grid->ny >= (int64_t(1) << 24))
        return fail(RTE_ERR_INVALID_ARG, "grid too large (%lld key points; limits: 2^27 key points, nx*ny < 2^24)",
                    (long long)nodes);
    if (ncams < 1) return fail(RTE_ERR_INVALID_ARG, "need at least one camera");
    const int W = cams[0].width, H = cams[0].height;
    if (W < 1 || H < 1) return fail(RTE_ERR_INVALID_ARG, "camera 0 has an empty image");
    for (int v = 0; v < ncams; ++v) {
        const rte_camera &c = cams[v];
        if (c.width != W || c.height != H)
            return fail(RTE_ERR_INVALID_ARG, "camera %d image size differs from camera 0", v);
        if (!std::isfinite(c.fx) || !std::isfinite(c.fy) || c.fx == 0.0 || c.fy == 0.0 ||
            !std::isfinite(c.cx) || !std::isfinite(c.cy))
            return fail(RTE_ERR_INVALID_ARG, "camera %d has invalid intrinsics", v);
        for (int i = 0; i < 9; ++i)
            if (!std::isfinite(c.R[i])) return fail(RTE_ERR_INVALID_ARG, "camera %d: R not finite", v);
        for (int i = 0; i < 3; ++i)
            if (!std::isfinite(c.t[i])) return fail(RTE_ERR_INVALID_ARG, "camera %d: t not finite", v);
    }
    const int C = params->channels;
    if (C != 1 && C != 3) return fail(RTE_ERR_INVALID_ARG, "channels must be 1 or 3 (got %d)", C);
    if ((int64_t)ncams * W * H * C >= (int64_t(1) << 31))
        return fail(RTE_ERR_INVALID_ARG, "images too large for 32-bit indexing");
    if (!finite_pos(params->step_vox)) return fail(RTE_ERR_INVALID_ARG, "step_vox must be > 0");
    if (!std::isfinite(params->albedo) || params->albedo < 0.0f)
        return fail(RTE_ERR_INVALID_ARG, "albedo must be >= 0");
    if (!std::isfinite(params->background))
        return fail(RTE_ERR_INVALID_ARG, "background must be finite");
    if (params->flags & ~RTE_PLAN_GRADIENTS) return fail(RTE_ERR_INVALID_ARG, "unknown plan flags 0x%x", params->flags);
    if (!(std::fabs(params->phase_g) < 1.0f)) return fail(RTE_ERR_INVALID_ARG, "phase_g must satisfy |g| < 1");
    if (params->albedo > 0.0f || params->scatter_res != 0) {
        if (params->scatter_res < 2 || params->scatter_res > 1024)
            return fail(RTE_ERR_INVALID_ARG, "scatter_res must be in [2, 1024] with albedo > 0");
        if (params->scatter_dirs < 1 || params->scatter_dirs > kMaxDirs)
            return fail(RTE_ERR_INVALID_ARG, "scatter_dirs must be in [1, %d]", kMaxDirs);
        if (!finite_pos(params->scatter_step))
            return fail(RTE_ERR_INVALID_ARG, "scatter_step must be > 0");
    }
    return RTE_OK;
}

struct Derived {
    int V, W, H, tiles_x, tiles_y, tiles_per_view, n_tiles;
    int64_t n_rays, n_nodes, n_cells, n_part_cells;
    double h[3], ds;
};

Derived derive(const rte_grid *grid, const rte_camera *cams, int32_t ncams, const rte_render_params *params)
{
    Derived d{};
    d.V = ncams;
    d.W = cams[0].width;
    d.H = cams[0].height;
    d.tiles_x = (d.W + rte::kTile - 1) / rte::kTile;
    d.tiles_y = (d.H + rte::kTile - 1) / rte::kTile;
    d.tiles_per_view = d.tiles_x * d.tiles_y;
    d.n_tiles = d.tiles_per_view * d.V;
    d.n_rays = (int64_t)d.V * d.W * d.H;
    d.n_nodes = (int64_t)grid->nx * grid->ny * grid->nz;
    d.n_cells = (int64_t)(grid->nx - 1) * (grid->ny - 1) * (grid->nz - 1);
    d.n_part_cells = (int64_t)((grid->nx - 1 + 7) / 8) * ((grid->ny - 1 + 7) / 8) * ((grid->nz - 1 + 3) / 4) * 256;
    const int n[3] = {grid->nx, grid->ny, grid->nz};
    double hmin = 1e300;
    for (int i = 0; i < 3; ++i) {
        d.h[i] = (grid->bbox_max[i] - grid->bbox_min[i]) / (double)(n[i] - 1);
        hmin = std::min(hmin, d.h[i]);
    }
    d.ds = (double)params->step_vox * hmin;
    return d;
}

// Rows of a tile in the per-sample buffers: its longest march rounded up to
// whole groups of four samples.
uint64_t group_rows(int kmax) { return ((uint64_t)kmax + rte::kGroup - 1) / rte::kGroup * rte::kGroup; }

// Host geometry of the tiles (same FP64 arithmetic as the device ray table):
// the per-tile maximum segment count, used for the workspace bound before any
// device work, and for the launch order each tile's sample count, the
// K-weighted sum of its rays' chord midpoints, and per axis the distance all
// samples travel along it.
struct HostTiles {
    std::vector<int> kmax;
    std::vector<double> work;       // samples (sum of K over the tile's rays)
    std::vector<double> mid[3];     // sum of K * chord midpoint, per axis
    double travel[3] = {0.0, 0.0, 0.0};
};

HostTiles host_tiles(const rte_grid *grid, const rte_camera *cams, const Derived &d)
{
    HostTiles h;
    h.kmax.assign(d.n_tiles, 0);
    h.work.assign(d.n_tiles, 0.0);
    for (auto &m : h.mid) m.assign(d.n_tiles, 0.0);
    for (int v = 0; v < d.V; ++v) {
        const rte_camera &c = cams[v];
        double o[3];
        for (int i = 0; i < 3; ++i) o[i] = -(c.R[0 * 3 + i] * c.t[0] + c.R[1 * 3 + i] * c.t[1] + c.R[2 * 3 + i] * c.t[2]);
        for (int py = 0; py < d.H; ++py)
            for (int px = 0; px < d.W; ++px) {
                const double dc0 = ((double)px + 0.5 - c.cx) / c.fx, dc1 = ((double)py + 0.5 - c.cy) / c.fy;
                double dir[3], n2 = 0.0;
                for (int i = 0; i < 3; ++i) {
                    dir[i] = c.R[0 * 3 + i] * dc0 + c.R[1 * 3 + i] * dc1 + c.R[2 * 3 + i];
                    n2 += dir[i] * dir[i];
                }
                const double inv = 1.0 / std::sqrt(n2);
                double t0 = -INFINITY, t1 = INFINITY;
                bool hit = true;
                for (int i = 0; i < 3; ++i) {
                    const double di = dir[i] * inv;
                    if (di != 0.0) {
                        double ta = (grid->bbox_min[i] - o[i]) / di, tb = (grid->bbox_max[i] - o[i]) / di;
                        if (ta > tb) std::swap(ta, tb);
                        t0 = std::max(t0, ta);
                        t1 = std::min(t1, tb);
                    } else if (o[i] < grid->bbox_min[i] || o[i] > grid->bbox_max[i]) {
                        hit = false;
                    }
                }
                t0 = std::max(t0, 0.0);
                if (!hit || !(t1 > t0)) continue;
                const int K = (int)std::ceil((t1 - t0) / d.ds);
                const size_t t = (size_t)v * d.tiles_per_view + (py / rte::kTile) * d.tiles_x + px / rte::kTile;
                h.kmax[t] = std::max(h.kmax[t], K);
                h.work[t] += K;
                for (int i = 0; i < 3; ++i) {
                    h.mid[i][t] += K * (o[i] + dir[i] * inv * 0.5 * (t0 + t1));
                    h.travel[i] += K * std::fabs(dir[i] * inv);
                }
            }
    }
    return h;
}

std::vector<int> host_tile_kmax(const rte_grid *grid, const rte_camera *cams, const Derived &d)
{
    return host_tiles(grid, cams, d).kmax;
}

// Launch slots of the render and the reverse march, four per block, block b
// running on XCD b mod 8. The tiles that hold samples are cut into 8 bands of
// equal sample count along the axis the samples travel least (for a ring of
// cameras around an axis, bands of height), band x going to XCD x, so that
// each XCD's L2 serves one band of the volume; each band runs its longest
// marches first, and a band that runs out of tiles before the longest band
// leaves its slots empty (-1; such a wave exits at once). The bands at the
// volume's ends hold more, shorter tiles than the middle ones (about 1.7x on
// a ring of cameras), so the slots come to about 1.4-1.6x the tiles; where
// they would exceed twice the tiles, one list, longest march first, is dealt
// to every XCD instead. Bands are used only for a packed volume of at most
// kBandVolumeBytes: one beyond the last-level cache (256 MB) is better served
// by every XCD marching the longest tiles, and so the same central part of
// the volume, at the same time (a 268 MB volume: reverse march 7.4 -> 9.4 ms
// with bands; a 33 MB one: render 0.655 -> 0.640 ms).
// Tiles without samples follow; they only receive the background in image
// renders. n_active: slots of the tiles with samples.
constexpr size_t kBandVolumeBytes = 64ull << 20;

std::vector<int32_t> tile_launch_order(const std::vector<int32_t> &kmax, const HostTiles &h, size_t vol_bytes,
                                       int &n_active)
{
    const int n = (int)kmax.size();
    auto longest = [&](int32_t a, int32_t b) { return kmax[a] > kmax[b]; };
    std::vector<int32_t> act;
    for (int t = 0; t < n; ++t)
        if (kmax[t] > 0) act.push_back(t);
    const int ax = (int)(std::min_element(h.travel, h.travel + 3) - h.travel);
    auto work = [&](int32_t t) { return h.work[t] > 0.0 ? h.work[t] : (double)kmax[t]; };
    auto key = [&](int32_t t) { return h.work[t] > 0.0 ? h.mid[ax][t] / h.work[t] : 0.0; };
    std::vector<int32_t> by_key = act;
    std::stable_sort(by_key.begin(), by_key.end(), [&](int32_t a, int32_t b) { return key(a) < key(b); });
    double total = 0.0;
    for (int32_t t : by_key) total += work(t);
    std::vector<std::vector<int32_t>> band(8);
    double run = 0.0;
    for (int32_t t : by_key) {
        band[std::min(7, (int)(8.0 * (run + 0.5 * work(t)) / std::max(total, 1.0)))].push_back(t);
        run += work(t);
    }
    size_t rounds = 0;
    for (auto &b : band) {
        std::stable_sort(b.begin(), b.end(), longest);
        rounds = std::max(rounds, (b.size() + 3) / 4);
    }
    std::vector<int32_t> order;
    if (vol_bytes <= kBandVolumeBytes && 32 * rounds <= 2 * act.size() + 32) {
        for (size_t i = 0; i < rounds; ++i)
            for (int x = 0; x < 8; ++x)
                for (size_t w = 0; w < 4; ++w) order.push_back(4 * i + w < band[x].size() ? band[x][4 * i + w] : -1);
    } else {
        order = act;
        std::stable_sort(order.begin(), order.end(), longest);
    }
    n_active = (int)order.size();
    for (int t = 0; t < n; ++t)
        if (kmax[t] == 0) order.push_back(t);
    return order;
}

// Launch slots a plan of n_tiles tiles can hold (see tile_launch_order).
int64_t max_slots(int64_t n_tiles) { return 2 * n_tiles + 32; }

struct Sizes {
    size_t cams, proj, rays, tnear, tiles, g, q, vol, scat, scat_part, dirs, dirs_world, y, part, cols, lut, mask,
        inside, err, total;
    int part_acc, lut_cap;
};

Sizes workspace(const rte_render_params *params, const Derived &d, uint64_t g_floats)
{
    Sizes s{};
    const int C = params->channels;
    const int M = params->scatter_res >= 2 ? params->scatter_res : 0;
    const bool grads = (params->flags & RTE_PLAN_GRADIENTS) != 0;
    // C + 1 accumulators per corner: room for a gather with column sums
    // (temperature fit, ordered subsets, gradients)
    s.part_acc = std::max(C + 1, 2);
    s.lut_cap = kMaxLut;
    s.cams = sizeof(rte_camera) * d.V;
    s.proj = sizeof(rte::ViewProj) * d.V;
    s.rays = 2 * sizeof(float4) * d.n_rays;
    s.tnear = sizeof(float) * d.n_rays;
    s.tiles = 3 * sizeof(int32_t) * d.n_tiles;
    s.g = sizeof(float) * std::max<uint64_t>(g_floats, 1);
    s.q = grads ? 2 * s.g : 0;  // (g_k, q_k) pairs of the adjoint march
    s.vol = (C == 3 ? 16 : 8) * (size_t)d.n_nodes;
    // one in-scatter grid per view for an anisotropic phase function
    const size_t grids = (M && params->phase_g != 0.0f) ? (size_t)d.V : 1;
    s.scat = sizeof(float4) * grids * std::max(M, 1) * std::max(M, 1) * std::max(M, 1);
    s.dirs = sizeof(float4) * kMaxDirs;
    s.dirs_world = 3 * sizeof(double) * kMaxDirs;
    // per-direction sums plus the slab-pass state (next sample, transmittance)
    s.scat_part = M ? sizeof(float) * (size_t)params->scatter_dirs * (C + 2) * M * M * M : sizeof(float);
    s.y = sizeof(float) * (size_t)d.n_rays * (C == 3 ? 4 : 1);  // per ray: float4 (RGB, pad) or float
    // back-projection partials: per gather brick, one plane of key points per
    // accumulator; the visual hull keeps two 32-bit view masks per cell there
    const int64_t bricks = std::max<int64_t>(d.n_part_cells / 256, 1);
    s.part = sizeof(float) * std::max<size_t>((size_t)s.part_acc * rte::kBrickNodeStride * bricks,
                                              2 * (size_t)std::max<int64_t>(d.n_part_cells, 1));
    s.cols = sizeof(float) * d.n_nodes;
    s.lut = sizeof(float) * 3 * (size_t)s.lut_cap;
    s.mask = sizeof(float) * (size_t)d.n_rays;
    s.inside = sizeof(int32_t) * (size_t)d.n_nodes;
    s.err = sizeof(float2) * (size_t)max_slots(d.n_tiles) + 2 * sizeof(double) + kBatchBytes;
    s.total = s.cams + s.proj + s.rays + s.tnear + s.tiles + s.g + s.q + s.vol + s.scat + s.scat_part + s.dirs +
              s.dirs_world +
              s.y + s.part + s.cols + s.lut + s.mask + s.inside + s.err;
    return s;
}

// ------------------------------------------------------------------ timing

hipEvent_t take_event(rte_plan *p);

// Timing events only measure: they skip the system-scope fence a default
// event performs when it is recorded (a cache writeback and invalidation that
// would also slow the launch after it).
hipEvent_t make_timing_event()
{
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
    return e;
}

// Adds the finished launches' times and returns their events to the pool;
// wait = false leaves launches still running in `pending` (no host wait).
void drain_timing(rte_plan *p, bool wait = true)
{
    size_t kept = 0;
    for (size_t i = 0; i < p->pending.size(); ++i) {
        const auto r = p->pending[i];
        if (!wait && hipEventQuery(r.stop) != hipSuccess) {
            p->pending[kept++] = r;
            continue;
        }
        float ms = 0.0f;
        if (hipEventSynchronize(r.stop) == hipSuccess && hipEventElapsedTime(&ms, r.start, r.stop) == hipSuccess) {
            p->kernel_ms[r.kernel] += ms;
            p->kernel_launches[r.kernel] += 1;
        }
        p->event_pool.push_back(r.start);
        p->event_pool.push_back(r.stop);
    }
    p->pending.resize(kept);
}

// An event for the next launch: from the pool, else from the launches that
// have finished, else a new one (the host never waits on the GPU here).
hipEvent_t take_event(rte_plan *p)
{
    if (p->event_pool.empty()) drain_timing(p, false);
    if (p->event_pool.empty()) return make_timing_event();
    hipEvent_t e = p->event_pool.back();
    p->event_pool.pop_back();
    return e;
}

// Brackets one launch with events when timing is enabled.
struct Timed {
    rte_plan *p;
    int kernel;
    hipStream_t s;
    hipEvent_t e0 = nullptr;
    Timed(rte_plan *p_, int k, hipStream_t s_) : p(p_), kernel(k), s(s_)
    {
        if ((p->timing_mask >> kernel) & 1u) {
            e0 = take_event(p);
            if (e0) hipEventRecord(e0, s);
        }
    }
    hipError_t done(hipError_t launch_status)
    {
        if (e0) {
            hipEvent_t e1 = take_event(p);
            if (e1) {
                hipEventRecord(e1, s);
                p->pending.push_back({kernel, e0, e1});
            }
        }
        return launch_status;
    }
};

#define RTE_LAUNCH(plan, kid, stream, call)                                               \
    do {                                                                                  \
        Timed t_((plan), (kid), (stream));                                                \
        hipError_t e_ = t_.done(call);                                                    \
        if (e_ != hipSuccess)                                                             \
            return fail(RTE_ERR_HIP, "launch of %s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

template <typename T>
int dev_alloc(T **ptr, size_t bytes, size_t &acc)
{
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) return fail(RTE_ERR_HIP, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    *ptr = static_cast<T *>(p);
    acc += bytes;
    return RTE_OK;
}

void free_plan(rte_plan *p)
{
    if (!p) return;
    hipDeviceSynchronize();
    for (auto &r : p->pending) {
        hipEventDestroy(r.start);
        hipEventDestroy(r.stop);
    }
    for (auto e : p->event_pool) hipEventDestroy(e);
    void *bufs[] = {p->d_cams, p->d_proj, p->d_rayA, p->d_rayB, p->d_tnear, p->d_tile_kmax,
                    p->d_tile_off, p->d_tile_order, p->d_g, p->d_q, p->d_vol, p->d_scat, p->d_scat_part, p->d_dirs, p->d_dirs_world, p->d_y, p->d_part,
                    p->d_cols, p->d_lut, p->d_mask, p->d_inside, p->d_err, p->d_err_sum};
    for (void *b : bufs)
        if (b) hipFree(b);
    if (p->h_err_sum) hipHostFree(p->h_err_sum);
    if (p->h_batch) hipHostFree(p->h_batch);
    if (p->batch_event) hipEventDestroy(p->batch_event);
    if (p->scat_event) hipEventDestroy(p->scat_event);
    if (p->d_batch) hipFree(p->d_batch);
    delete p;
}

// Voxel-coordinate -> homogeneous pixel projection of each view.
rte::ViewProj view_projection(const rte_grid *g, const rte_camera &c, const double h[3])
{
    // x_w = lo + h * X ; x_c = R x_w + t ; (hu, hv, hw) = (fx xc + cx zc, fy yc + cy zc, zc)
    double Rh[3][4];
    for (int r = 0; r < 3; ++r) {
        for (int k = 0; k < 3; ++k) Rh[r][k] = c.R[r * 3 + k] * h[k];
        Rh[r][3] = c.R[r * 3 + 0] * g->bbox_min[0] + c.R[r * 3 + 1] * g->bbox_min[1] +
                   c.R[r * 3 + 2] * g->bbox_min[2] + c.t[r];
    }
    rte::ViewProj vp{};
    for (int k = 0; k < 4; ++k) {
        vp.P[0 + k] = (float)(c.fx * Rh[0][k] + c.cx * Rh[2][k]);
        vp.P[4 + k] = (float)(c.fy * Rh[1][k] + c.cy * Rh[2][k]);
        vp.P[8 + k] = (float)Rh[2][k];
    }
    return vp;
}

int check_plan(const rte_plan *p)
{
    if (!p) return fail(RTE_ERR_INVALID_ARG, "null plan");
    return RTE_OK;
}

int ensure_lut(rte_plan *p, const rte_temp_params *tp, hipStream_t s)
{
    if (!tp) return fail(RTE_ERR_INVALID_ARG, "null temperature params");
    if (tp->lut_size < 2 || tp->lut_size > p->lut_cap)
        return fail(RTE_ERR_INVALID_ARG, "lut_size must be in [2, %d]", p->lut_cap);
    if (!(tp->t_max > tp->t_min) || !(tp->t_min > 0.0f) || !std::isfinite(tp->t_max) || !(tp->t_norm > 0.0f))
        return fail(RTE_ERR_INVALID_ARG, "temperature range invalid");
    if (!finite_pos(tp->band_std_nm)) return fail(RTE_ERR_INVALID_ARG, "band_std_nm must be > 0");
    for (int c = 0; c < 3; ++c)
        if (!finite_pos(tp->band_nm[c]) || (double)tp->band_nm[c] - 6.0 * (double)tp->band_std_nm <= 0.0)
            return fail(RTE_ERR_INVALID_ARG, "band %d must lie at positive wavelengths", c);
    if (tp->channel < 0 || tp->channel > 2) return fail(RTE_ERR_INVALID_ARG, "channel must be 0, 1 or 2");
    if (!(tp->soot_span > 0.0f) || !std::isfinite(tp->sigma_max) || tp->sigma_max < 0.0f)
        return fail(RTE_ERR_INVALID_ARG, "soot_span must be > 0 and sigma_max >= 0");
    if (tp->panels < 2 || tp->panels > (1 << 20)) return fail(RTE_ERR_INVALID_ARG, "panels out of range");
    if (p->lut_valid && std::memcmp(&p->lut_params, tp, sizeof(*tp)) == 0) return RTE_OK;
    rte::build_temperature_lut(*tp, p->lut_host);
    for (int i = 1; i < tp->lut_size; ++i)
        if (!(p->lut_host[(size_t)tp->channel * tp->lut_size + i] >
              p->lut_host[(size_t)tp->channel * tp->lut_size + i - 1]))
            return fail(RTE_ERR_INVALID_ARG, "fitted channel is not increasing in temperature on [t_min, t_max]");
    for (int c = 0; c < 3; ++c)
        RTE_HIP(hipMemcpyAsync(p->d_lut + (size_t)c * p->lut_cap, p->lut_host.data() + (size_t)c * tp->lut_size,
                               sizeof(float) * tp->lut_size, hipMemcpyHostToDevice, s));
    RTE_HIP(hipStreamSynchronize(s));
    p->lut_params = *tp;
    p->lut_valid = true;
    return RTE_OK;
}

}  // namespace

extern "C" {

const char *rte_last_error(void) { return g_last_error.c_str(); }

size_t rte_plan_workspace_bytes(const rte_grid *grid, const rte_camera *cams, int32_t ncams,
                                const rte_render_params *params)
{
    if (validate_config(grid, cams, ncams, params) != RTE_OK) return 0;
    const Derived d = derive(grid, cams, ncams, params);
    const std::vector<int> kmax = host_tile_kmax(grid, cams, d);
    uint64_t g = 0;
    for (int k : kmax) g += (uint64_t)group_rows(k + 1) * rte::kTileRays;
    return workspace(params, d, g).total;
}

int rte_plan_create(rte_plan **out, const rte_grid *grid, const rte_camera *cams, int32_t ncams,
                    const rte_render_params *params, size_t hbm_budget_bytes, void *stream)
{
    if (!out) return fail(RTE_ERR_INVALID_ARG, "null output pointer");
    *out = nullptr;
    int rc = validate_config(grid, cams, ncams, params);
    if (rc) return rc;
    const Derived d = derive(grid, cams, ncams, params);
    const HostTiles host = host_tiles(grid, cams, d);
    const std::vector<int> &host_kmax = host.kmax;
    uint64_t g_bound = 0;
    for (int k : host_kmax) g_bound += (uint64_t)group_rows(k + 1) * rte::kTileRays;
    const Sizes bound = workspace(params, d, g_bound);
    if (hbm_budget_bytes && bound.total > hbm_budget_bytes)
        return fail(RTE_ERR_BUDGET, "plan needs up to %zu bytes, budget is %zu", bound.total, hbm_budget_bytes);

    hipStream_t s = static_cast<hipStream_t>(stream);
    rte_plan *p = new rte_plan();
    p->grid = *grid;
    p->params = *params;
    p->cams.assign(cams, cams + ncams);
    p->V = d.V;
    p->W = d.W;
    p->H = d.H;
    p->tiles_x = d.tiles_x;
    p->tiles_y = d.tiles_y;
    p->tiles_per_view = d.tiles_per_view;
    p->n_tiles = d.n_tiles;
    p->n_rays = d.n_rays;
    p->n_nodes = d.n_nodes;
    p->n_cells = d.n_cells;
    p->n_part_cells = d.n_part_cells;
    for (int i = 0; i < 3; ++i) p->h[i] = d.h[i];
    p->ds = d.ds;
    p->last_stream = s;
    auto bail = [&](int code) {
        std::string msg = g_last_error;
        free_plan(p);
        g_last_error = msg;
        return code;
    };

    // ray table (K4) and per-tile maxima
    size_t acc = 0;
    const Sizes sz = workspace(params, d, 0);
    if ((rc = dev_alloc(&p->d_cams, sz.cams, acc)) || (rc = dev_alloc(&p->d_proj, sz.proj, acc)) ||
        (rc = dev_alloc(&p->d_rayA, sz.rays / 2, acc)) || (rc = dev_alloc(&p->d_rayB, sz.rays / 2, acc)) ||
        (rc = dev_alloc(&p->d_tnear, sz.tnear, acc)) ||
        (rc = dev_alloc(&p->d_tile_kmax, sizeof(int32_t) * d.n_tiles, acc)) ||
        (rc = dev_alloc(&p->d_tile_off, sizeof(uint32_t) * d.n_tiles, acc)))
        return bail(rc);
    std::vector<rte::ViewProj> proj(d.V);
    for (int v = 0; v < d.V; ++v) proj[v] = view_projection(grid, cams[v], d.h);
    if (hipMemcpyAsync(p->d_cams, cams, sz.cams, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(p->d_proj, proj.data(), sz.proj, hipMemcpyHostToDevice, s) != hipSuccess)
        return bail(fail(RTE_ERR_HIP, "camera upload failed"));
    {
        Timed t(p, RTE_KERNEL_RAYS, s);
        hipError_t e = t.done(rte::launch_ray_table(p, s));
        if (e == hipSuccess) e = rte::launch_tile_kmax(p, s);
        if (e != hipSuccess) return bail(fail(RTE_ERR_HIP, "ray table launch failed: %s", hipGetErrorString(e)));
    }
    std::vector<int32_t> kmax(d.n_tiles);
    if (hipMemcpyAsync(kmax.data(), p->d_tile_kmax, sizeof(int32_t) * d.n_tiles, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return bail(fail(RTE_ERR_HIP, "ray table readback failed"));
    std::vector<uint32_t> off(d.n_tiles);
    uint64_t g = 0;
    for (int t = 0; t < d.n_tiles; ++t) {
        if (kmax[t] > host_kmax[t] + 1)
            return bail(fail(RTE_ERR_HIP, "device ray table disagrees with the host bound at tile %d", t));
        off[t] = (uint32_t)g;
        g += (uint64_t)group_rows(kmax[t]) * rte::kTileRays;
    }
    if (g > 0xFFFFFFFFull)
        return bail(fail(RTE_ERR_UNSUPPORTED, "%llu per-sample slots exceed the 2^32 a plan addresses; use fewer views "
                                              "or a coarser step", (unsigned long long)g));
    p->g_floats = g;
    // launch order of the render and the reverse march
    const size_t vol_bytes = (params->channels == 3 ? 16 : 8) * (size_t)d.n_nodes;
    const std::vector<int32_t> order = tile_launch_order(kmax, host, vol_bytes, p->n_active_slots);
    p->n_slots = (int)order.size();
    if ((rc = dev_alloc(&p->d_tile_order, sizeof(int32_t) * std::max<size_t>(order.size(), 1), acc)))
        return bail(rc);
    if (hipMemcpyAsync(p->d_tile_off, off.data(), sizeof(uint32_t) * d.n_tiles, hipMemcpyHostToDevice, s) != hipSuccess ||
        (!order.empty() && hipMemcpyAsync(p->d_tile_order, order.data(), sizeof(int32_t) * order.size(),
                                          hipMemcpyHostToDevice, s) != hipSuccess))
        return bail(fail(RTE_ERR_HIP, "tile tables upload failed"));

    // remaining workspaces
    const Sizes full = workspace(params, d, g);
    const int M = params->scatter_res >= 2 ? params->scatter_res : 0;
    p->part_acc = full.part_acc;
    p->lut_cap = full.lut_cap;
    if ((rc = dev_alloc(&p->d_g, full.g, acc)) || (full.q && (rc = dev_alloc(&p->d_q, full.q, acc))) ||
        (rc = dev_alloc(&p->d_vol, full.vol, acc)) ||
        (rc = dev_alloc(&p->d_scat, full.scat, acc)) || (rc = dev_alloc(&p->d_scat_part, full.scat_part, acc)) ||
        (rc = dev_alloc(&p->d_dirs, full.dirs, acc)) || (rc = dev_alloc(&p->d_dirs_world, full.dirs_world, acc)) ||
        (rc = dev_alloc(&p->d_y, full.y, acc)) || (rc = dev_alloc(&p->d_part, full.part, acc)) ||
        (rc = dev_alloc(&p->d_cols, full.cols, acc)) || (rc = dev_alloc(&p->d_lut, full.lut, acc)) ||
        (rc = dev_alloc(&p->d_mask, full.mask, acc)) || (rc = dev_alloc(&p->d_inside, full.inside, acc)) ||
        (rc = dev_alloc(&p->d_err, sizeof(float2) * (size_t)p->n_slots, acc)) ||
        (rc = dev_alloc(&p->d_err_sum, 2 * sizeof(double), acc)))
        return bail(rc);
    if ((rc = dev_alloc(&p->d_batch, kBatchBytes, acc))) return bail(rc);
    p->batch_bytes = kBatchBytes - kScatStageBytes;
    p->scat_stage_off = kBatchBytes - kScatStageBytes;
    p->scat_stage_bytes = kScatStageBytes;
    if (hipHostMalloc((void **)&p->h_err_sum, 2 * sizeof(double), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(&p->h_batch, kBatchBytes, hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&p->batch_event, hipEventDisableTiming) != hipSuccess ||
        hipEventRecord(p->batch_event, s) != hipSuccess ||
        hipEventCreateWithFlags(&p->scat_event, hipEventDisableTiming) != hipSuccess ||
        hipEventRecord(p->scat_event, s) != hipSuccess)
        return bail(fail(RTE_ERR_HIP, "pinned host allocation failed"));
    // in-scatter directions: spherical Fibonacci, voxel units per world unit
    if (M) {
        std::vector<float4> dirs(kMaxDirs, make_float4(0.f, 0.f, 0.f, 0.f));
        std::vector<double> world(3 * kMaxDirs, 0.0);
        const int nd = params->scatter_dirs;
        for (int k = 0; k < nd; ++k) {
            const double z = 1.0 - (2.0 * k + 1.0) / (double)nd;
            const double r = std::sqrt(std::max(0.0, 1.0 - z * z));
            const double ph = (double)k * M_PI * (3.0 - std::sqrt(5.0));
            world[3 * k] = r * std::cos(ph);
            world[3 * k + 1] = r * std::sin(ph);
            world[3 * k + 2] = z;
            dirs[k] = make_float4((float)(world[3 * k] / d.h[0]), (float)(world[3 * k + 1] / d.h[1]),
                                  (float)(z / d.h[2]), 0.f);
        }
        // z decreases with k: the upward directions come first
        p->scat_nup = 0;
        while (p->scat_nup < nd && dirs[p->scat_nup].z >= 0.0f) ++p->scat_nup;
        if (hipMemcpyAsync(p->d_dirs, dirs.data(), full.dirs, hipMemcpyHostToDevice, s) != hipSuccess ||
            hipMemcpyAsync(p->d_dirs_world, world.data(), full.dirs_world, hipMemcpyHostToDevice, s) != hipSuccess ||
            hipMemsetAsync(p->d_scat, 0, full.scat, s) != hipSuccess)
            return bail(fail(RTE_ERR_HIP, "in-scatter setup failed"));
    }
    if (hipStreamSynchronize(s) != hipSuccess) return bail(fail(RTE_ERR_HIP, "plan setup sync failed"));
    uint64_t samples = 0, hits = 0;
    {
        // exact counts from the device ray table
        std::vector<float4> B(d.n_rays);
        if (hipMemcpy(B.data(), p->d_rayB, sizeof(float4) * d.n_rays, hipMemcpyDeviceToHost) != hipSuccess)
            return bail(fail(RTE_ERR_HIP, "ray table count readback failed"));
        for (const float4 &b : B) {
            int K;
            std::memcpy(&K, &b.w, sizeof(int));
            samples += (uint64_t)K;
            hits += K > 0;
        }
    }
    p->samples = samples;
    p->hit_rays = hits;
    p->device_bytes = acc;
    *out = p;
    return ok();
}

size_t rte_plan_device_bytes(const rte_plan *plan) { return plan ? plan->device_bytes : 0; }

void rte_plan_destroy(rte_plan *plan) { free_plan(plan); }

int rte_suggest_grid(const rte_camera *cams, int32_t ncams, const double bbox_min[3], const double bbox_max[3],
                     double alpha, rte_grid *grid, double *n_max)
{
    if (!cams || !bbox_min || !bbox_max || !grid) return fail(RTE_ERR_INVALID_ARG, "null argument");
    if (ncams < 1) return fail(RTE_ERR_INVALID_ARG, "need at least one camera");
    if (!(alpha > 0.0) || !std::isfinite(alpha)) return fail(RTE_ERR_INVALID_ARG, "alpha must be > 0");
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(bbox_min[a]) || !std::isfinite(bbox_max[a]) || !(bbox_max[a] > bbox_min[a]))
            return fail(RTE_ERR_INVALID_ARG, "bbox axis %d is empty or not finite", a);
    double span[3] = {0.0, 0.0, 0.0};
    for (int v = 0; v < ncams; ++v) {
        const rte_camera &c = cams[v];
        // corner index bits: x (1), y (2), z (4); camera coordinates of each
        double pc[8][3];
        for (int k = 0; k < 8; ++k) {
            const double w[3] = {(k & 1) ? bbox_max[0] : bbox_min[0], (k & 2) ? bbox_max[1] : bbox_min[1],
                                 (k & 4) ? bbox_max[2] : bbox_min[2]};
            for (int r = 0; r < 3; ++r) pc[k][r] = c.R[3 * r] * w[0] + c.R[3 * r + 1] * w[1] + c.R[3 * r + 2] * w[2] + c.t[r];
        }
        for (int axis = 0; axis < 3; ++axis) {
            const int bit = 1 << axis;
            for (int k = 0; k < 8; ++k) {
                if (k & bit) continue;
                const double *p0 = pc[k], *p1 = pc[k | bit];
                if (!(p0[2] > 0.0) || !(p1[2] > 0.0)) continue;  // crosses or lies behind the image plane
                const double du = std::fabs((c.fx * (p1[0] / p1[2]) + c.cx) - (c.fx * (p0[0] / p0[2]) + c.cx));
                const double dv = std::fabs((c.fy * (p1[1] / p1[2]) + c.cy) - (c.fy * (p0[1] / p0[2]) + c.cy));
                span[axis] = std::max(span[axis], std::max(du, dv));
            }
        }
    }
    int32_t nodes[3];
    for (int a = 0; a < 3; ++a) {
        if (!(span[a] > 0.0)) return fail(RTE_ERR_INVALID_ARG, "no edge along axis %d projects into any view", a);
        const double vox = std::ceil(span[a] / alpha);
        if (vox > 65535.0) return fail(RTE_ERR_INVALID_ARG, "axis %d would need %.0f voxels", a, vox);
        nodes[a] = (int32_t)std::max(vox, 1.0) + 1;
    }
    grid->nx = nodes[0];
    grid->ny = nodes[1];
    grid->nz = nodes[2];
    for (int a = 0; a < 3; ++a) {
        grid->bbox_min[a] = bbox_min[a];
        grid->bbox_max[a] = bbox_max[a];
        if (n_max) n_max[a] = span[a];
    }
    return ok();
}

int rte_plan_counts(const rte_plan *plan, uint64_t *samples, uint64_t *hit_rays)
{
    if (int rc = check_plan(plan)) return rc;
    if (samples) *samples = plan->samples;
    if (hit_rays) *hit_rays = plan->hit_rays;
    return ok();
}

int rte_ray_table(rte_plan *plan, float *t_near, float *t_far, int32_t *nseg, void *stream)
{
    if (int rc = check_plan(plan)) return rc;
    if (!t_near && !t_far && !nseg) return fail(RTE_ERR_INVALID_ARG, "no output requested");
    hipStream_t s = static_cast<hipStream_t>(stream);
    plan->last_stream = s;
    RTE_LAUNCH(plan, RTE_KERNEL_RAYS, s, rte::launch_ray_export(plan, t_near, t_far, nseg, s));
    return ok();
}

int rte_render(rte_plan *plan, const float *emission, const float *extinction, const float *inscatter,
               float *images, void *stream)
{
    if (int rc = check_plan(plan)) return rc;
    if (!emission || !extinction || !images) return fail(RTE_ERR_INVALID_ARG, "null emission, extinction or images");
    hipStream_t s = static_cast<hipStream_t>(stream);
    plan->last_stream = s;
    const int C = plan->params.channels;
    const bool scat = inscatter && plan->params.albedo > 0.0f && plan->params.scatter_res >= 2;
    RTE_LAUNCH(plan, RTE_KERNEL_PACK, s, rte::launch_pack(plan, emission, extinction, C, s));
    if (scat) RTE_LAUNCH(plan, RTE_KERNEL_PACK, s, rte::launch_pack_scatter(plan, inscatter, s));
    RTE_LAUNCH(plan, RTE_KERNEL_RENDER, s,
               rte::launch_render(plan, C, true, scat, false, rte::kEpiImage, nullptr, C, 0, images, s));
    return ok();
}

int rte_render_static(const rte_grid *grid, const rte_camera *cams, int32_t ncams,
                      const rte_render_params *params, const float *emission, const float *extinction,
                      const float *inscatter, float *images, void *stream)
{
    int rc = validate_config(grid, cams, ncams, params);
    if (rc) return rc;
    if (!emission || !extinction || !images) return fail(RTE_ERR_INVALID_ARG, "null emission, extinction or images");
    if (ncams > rte::kStaticMaxViews)
        return fail(RTE_ERR_UNSUPPORTED, "rte_render_static takes at most %d cameras (got %d)",
                    rte::kStaticMaxViews, ncams);
    const Derived d = derive(grid, cams, ncams, params);
    const int M = params->scatter_res >= 2 ? params->scatter_res : 0;
    const rte::StaticLayout L =
        rte::static_layout(d.V, d.W, d.H, d.n_nodes, params->channels, M, params->phase_g != 0.0f);
    if (L.total > rte::kStaticScratchBytes)
        return fail(RTE_ERR_BUDGET,
                    "rte_render_static needs %zu bytes of workspace; its static device array holds %zu "
                    "(use a plan: rte_plan_create + rte_render)",
                    L.total, rte::kStaticScratchBytes);
    // a plan that owns nothing: its configuration, with workspace pointers
    // that the launcher sets into the static array
    rte_plan view;
    view.grid = *grid;
    view.params = *params;
    view.V = d.V;
    view.W = d.W;
    view.H = d.H;
    view.tiles_x = d.tiles_x;
    view.tiles_y = d.tiles_y;
    view.tiles_per_view = d.tiles_per_view;
    view.n_tiles = d.n_tiles;
    view.n_rays = d.n_rays;
    view.n_nodes = d.n_nodes;
    view.n_cells = d.n_cells;
    view.n_part_cells = d.n_part_cells;
    for (int i = 0; i < 3; ++i) view.h[i] = d.h[i];
    view.ds = d.ds;
    const hipError_t e = rte::launch_render_static(&view, cams, emission, extinction, inscatter, images,
                                                   static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return fail(RTE_ERR_HIP, "rte_render_static launch failed: %s", hipGetErrorString(e));
    return ok();
}

int rte_render_forward(rte_plan *plan, const float *emission, const float *extinction, const float *inscatter,
                       float *images, double *exit_optical_depth, void *stream)
{
    if (int rc = check_plan(plan)) return rc;
    if (!emission || !extinction || !images || !exit_optical_depth)
        return fail(RTE_ERR_INVALID_ARG, "null emission, extinction, images or exit optical depth");
    hipStream_t s = static_cast<hipStream_t>(stream);
    plan->last_stream = s;
    const int C = plan->params.channels;
    const bool scat = inscatter && plan->params.albedo > 0.0f && plan->params.scatter_res >= 2;
    RTE_LAUNCH(plan, RTE_KERNEL_PACK, s, rte::launch_pack(plan, emission, extinction, C, s));
    if (scat) RTE_LAUNCH(plan, RTE_KERNEL_PACK, s, rte::launch_pack_scatter(plan, inscatter, s));
    RTE_LAUNCH(plan, RTE_KERNEL_RENDER, s,
               rte::launch_render(plan, C, true, scat, false, rte::kEpiImage, nullptr, C, 0, images, s,
                                  exit_optical_depth));
    return ok();
}

int rte_render_backward(rte_plan *plan, const float *emission, const float *extinction, const float *inscatter,
                        const double *exit_optical_depth, const float *grad_images, float *grad_emission,
                        float *grad_extinction, void *stream)
{
    if (int rc = check_plan(plan)) return rc;
    if (!(plan->params.flags & RTE_PLAN_GRADIENTS) || !plan->d_q)
        return fail(RTE_ERR_UNSUPPORTED, "plan was created without RTE_PLAN_GRADIENTS");
    if (!emission || !extinction || !exit_optical_depth || !grad_images || !grad_emission || !grad_extinction)
        return fail(RTE_ERR_INVALID_ARG, "null argument");
    hipStream_t s = static_cast<hipStream_t>(stream);
    plan->last_stream = s;
    const int C = plan->params.channels;
    const bool scat = inscatter && plan->params.albedo > 0.0f && plan->params.scatter_res >= 2;
    RTE_LAUNCH(plan, RTE_KERNEL_PACK, s, rte::launch_pack(plan, emission, extinction, C, s));
    if (scat) RTE_LAUNCH(plan, RTE_KERNEL_PACK, s, rte::launch_pack_scatter(plan, inscatter, s));
    RTE_LAUNCH(plan, RTE_KERNEL_ADJOINT, s, rte::launch_adjoint_march(plan, scat, exit_optical_depth, grad_images, s));
    const float *dI = nullptr;
    RTE_LAUNCH(plan, RTE_KERNEL_PACK, s, rte::launch_pack_residual(plan, grad_images, &dI, s));
    RTE_LAUNCH(plan, RTE_KERNEL_GATHER, s, rte::launch_gather(plan, C, rte::kGatherGrad, dI, 0.f, 0.f, 0.f, s));
    RTE_LAUNCH(plan, RTE_KERNEL_UPDATE, s,
               rte::launch_update(plan, C, C + 1, rte::kUpdGrad, 0.f, 0, grad_emission, nullptr, 0, 0, s,
                                  grad_extinction));
    return ok();
}

int rte_inscatter(rte_plan *plan, const float *emission, const float *extinction, float *inscatter, void *stream)
{
    if (int rc = check_plan(plan)) return rc;
    if (!emission || !extinction || !inscatter) return fail(RTE_ERR_INVALID_ARG, "null emission, extinction or output");
    if (plan->params.scatter_res < 2)
        return fail(RTE_ERR_UNSUPPORTED, "plan was created without an in-scatter grid (scatter_res < 2)");
    hipStream_t s = static_cast<hipStream_t>(stream);
    plan->last_stream = s;
    const int C = plan->params.channels;
    RTE_LAUNCH(plan, RTE_KERNEL_PACK, s, rte::launch_pack(plan, emission, extinction, C, s));
    RTE_LAUNCH(plan, RTE_KERNEL_INSCATTER, s, rte::launch_inscatter(plan, inscatter, s));
    return ok();
}

int rte_backproject(rte_plan *plan, const float *extinction, const float *residual, float *delta,
                    int32_t mode, const rte_recon_params *params, void *stream)
{
    if (int rc = check_plan(plan)) return rc;
    if (!residual || !delta) return fail(RTE_ERR_INVALID_ARG, "null residual or delta");
    if (mode != RTE_BP_ADJOINT && mode != RTE_BP_PAPER) return fail(RTE_ERR_INVALID_ARG, "unknown back-projection mode %d", mode);
    if (mode == RTE_BP_ADJOINT && !extinction) return fail(RTE_ERR_INVALID_ARG, "adjoint back-projection needs the extinction");
    if (mode == RTE_BP_PAPER && !params) return fail(RTE_ERR_INVALID_ARG, "paper back-projection needs alpha_l, alpha_d, tau");
    if (mode == RTE_BP_PAPER && !(params->tau >= 0.0f && params->tau < 1.0f))
        return fail(RTE_ERR_INVALID_ARG, "tau must be in [0, 1)");
    hipStream_t s = static_cast<hipStream_t>(stream);
    plan->last_stream = s;
    const int C = plan->params.channels;
    const float *y = nullptr;
    RTE_LAUNCH(plan, RTE_KERNEL_PACK, s, rte::launch_pack_residual(plan, residual, &y, s));
    if (mode == RTE_BP_ADJOINT) {
        RTE_LAUNCH(plan, RTE_KERNEL_PACK, s, rte::launch_pack(plan, nullptr, extinction, C, s));
        RTE_LAUNCH(plan, RTE_KERNEL_WEIGHTS, s,
                   rte::launch_render(plan, C, false, false, true, -1, nullptr, C, 0, nullptr, s));
        RTE_LAUNCH(plan, RTE_KERNEL_GATHER, s, rte::launch_gather(plan, C, rte::kGatherAdjoint, y, 0.f, 0.f, 0.f, s));
    } else {
        RTE_LAUNCH(plan, RTE_KERNEL_GATHER, s,
                   rte::launch_gather(plan, C, rte::kGatherPaper, y, params->alpha_l, params->alpha_d, params->tau, s));
    }
    RTE_LAUNCH(plan, RTE_KERNEL_UPDATE, s,
               rte::launch_update(plan, C, C, rte::kUpdDelta, 0.f, 0, delta, nullptr, 0, 0, s));
    return ok();
}

int rte_reconstruct(rte_plan *plan, const float *frames, const float *extinction, float *emission,
                    int32_t iters, const rte_recon_params *params, void *stream)
{
    if (int rc = check_plan(plan)) return rc;
    if (!frames || !extinction || !emission || !params)
        return fail(RTE_ERR_INVALID_ARG, "null frames, extinction, emission or params");
    if (iters < 0) return fail(RTE_ERR_INVALID_ARG, "iters must be >= 0");
    const int upd = params->update;
    if (upd != RTE_UPDATE_SART && upd != RTE_UPDATE_PAPER && upd != RTE_UPDATE_MLEM)
        return fail(RTE_ERR_INVALID_ARG, "unknown update rule %d", upd);
    if (!std::isfinite(params->lambda)) return fail(RTE_ERR_INVALID_ARG, "lambda must be finite");
    if (upd == RTE_UPDATE_PAPER && !(params->tau >= 0.0f && params->tau < 1.0f))
        return fail(RTE_ERR_INVALID_ARG, "tau must be in [0, 1)");
    if (!(params->g_sigma >= 0.0f) || !std::isfinite(params->g_sigma))
        return fail(RTE_ERR_INVALID_ARG, "g_sigma must be finite and >= 0");
    if (params->use_hull && plan->V > 64) return fail(RTE_ERR_UNSUPPORTED, "the visual hull supports at most 64 views");
    if (!(params->stop_tol >= 0.0f)) return fail(RTE_ERR_INVALID_ARG, "stop_tol must be >= 0");
    const int nsub = std::max(1, (int)params->ordered_subsets);
    if (nsub > plan->V) return fail(RTE_ERR_INVALID_ARG, "ordered_subsets (%d) exceeds the views (%d)", nsub, plan->V);
    if (nsub > 1 && (params->stop_tol > 0.0f || params->g_sigma != 0.0f))
        return fail(RTE_ERR_UNSUPPORTED, "ordered subsets are not combined with the stop rule or the gains G(s)");
    hipStream_t s = static_cast<hipStream_t>(stream);
    plan->last_stream = s;
    plan->last_iters = 0;
    plan->last_errors.clear();
    const int C = plan->params.channels;
    const bool scat = plan->params.albedo > 0.0f && plan->params.scatter_res >= 2;
    const float *mask = params->use_mask ? plan->d_mask : nullptr;
    const int32_t *inside = params->use_hull ? plan->d_inside : nullptr;
    const bool stop = params->stop_tol > 0.0f;
    RTE_LAUNCH(plan, RTE_KERNEL_PACK, s, rte::launch_pack(plan, emission, extinction, C, s));
    if (params->use_mask)
        RTE_LAUNCH(plan, RTE_KERNEL_PACK, s,
                   rte::launch_flame_mask(plan, frames, C, params->flame_threshold, plan->d_mask, s));
    if (params->use_hull) {
        RTE_LAUNCH(plan, RTE_KERNEL_GATHER, s, rte::launch_hull(plan, mask, plan->d_inside, s));
        RTE_LAUNCH(plan, RTE_KERNEL_UPDATE, s,
                   rte::launch_apply_outside(plan, C, plan->d_inside, params->outside_value, s));
    }
    // SART and EM: the per-sample weights g depend on the extinction only, so
    // the first iteration's render stores them for every later gather; row
    // sums come out of every render; column sums A^T 1 (over the adjusted
    // rays) come out of the first iteration's gather (stored for the later
    // iterations), or per subset along with each subset's gather
    const bool weights = upd != RTE_UPDATE_PAPER;
    const int epi = upd == RTE_UPDATE_SART ? rte::kEpiSart : (upd == RTE_UPDATE_MLEM ? rte::kEpiMlem : rte::kEpiPaper);
    if (nsub > 1) {
        // ordered subsets: view v in subset v mod nsub; one update per subset
        const bool paper = upd == RTE_UPDATE_PAPER;
        const int gmode = paper ? rte::kGatherPaper : rte::kGatherAdjointCols;
        const int umode = paper ? rte::kUpdPaper : (upd == RTE_UPDATE_SART ? rte::kUpdSartOS : rte::kUpdMlemOS);
        const int acc = paper ? C : C + 1;
        for (int it = 0; it < iters; ++it) {
            if (scat) RTE_LAUNCH(plan, RTE_KERNEL_INSCATTER, s, rte::launch_inscatter(plan, nullptr, s));
            for (int sb = 0; sb < nsub; ++sb) {
                RTE_LAUNCH(plan, RTE_KERNEL_RENDER, s,
                           rte::launch_render(plan, C, true, scat, weights && it == 0, epi, frames, C, 0, plan->d_y,
                                              s, nullptr, mask, nullptr, nsub, sb));
                RTE_LAUNCH(plan, RTE_KERNEL_GATHER, s,
                           rte::launch_gather(plan, C, gmode, plan->d_y, params->alpha_l, params->alpha_d, params->tau,
                                              s, paper ? nullptr : mask, 0.f, 0, it, sb, nsub));
                RTE_LAUNCH(plan, RTE_KERNEL_UPDATE, s,
                           rte::launch_update(plan, C, acc, umode, params->lambda, params->clamp_nonneg, nullptr,
                                              nullptr, 0, 0, s, nullptr, inside));
            }
            plan->last_iters = it + 1;
        }
        RTE_LAUNCH(plan, RTE_KERNEL_PACK, s, rte::launch_unpack(plan, emission, C, s));
        return ok();
    }
    const int gmode = upd == RTE_UPDATE_PAPER ? rte::kGatherPaper : rte::kGatherAdjoint;
    const int umode = upd == RTE_UPDATE_SART ? rte::kUpdSart : (upd == RTE_UPDATE_MLEM ? rte::kUpdMlem : rte::kUpdPaper);
    double prev_err = 0.0;
    for (int it = 0; it < iters; ++it) {
        if (scat) RTE_LAUNCH(plan, RTE_KERNEL_INSCATTER, s, rte::launch_inscatter(plan, nullptr, s));
        RTE_LAUNCH(plan, RTE_KERNEL_RENDER, s,
                   rte::launch_render(plan, C, true, scat, weights && it == 0, epi, frames, C, 0, plan->d_y, s,
                                      nullptr, mask, stop ? plan->d_err : nullptr));
        if (stop) {
            RTE_LAUNCH(plan, RTE_KERNEL_UPDATE, s, rte::launch_err_reduce(plan, plan->d_err_sum, s));
            RTE_HIP(hipMemcpyAsync(plan->h_err_sum, plan->d_err_sum, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
            RTE_HIP(hipStreamSynchronize(s));
            const double cnt = plan->h_err_sum[1];
            const double err = cnt > 0.0 ? std::sqrt(plan->h_err_sum[0] / cnt) : 0.0;
            plan->last_errors.push_back((float)err);
            if (it >= 1 && std::fabs(prev_err - err) < (double)params->stop_tol) break;
            prev_err = err;
        }
        if (it == 0 && upd != RTE_UPDATE_PAPER) {
            // the first gather also accumulates the column sums (over the
            // adjusted rays: masked rays are skipped, their residual is 0);
            // the update uses them and keeps them for the later iterations
            RTE_LAUNCH(plan, RTE_KERNEL_GATHER, s,
                       rte::launch_gather(plan, C, rte::kGatherAdjointCols, plan->d_y, 0.f, 0.f, 0.f, s, mask));
            RTE_LAUNCH(plan, RTE_KERNEL_UPDATE, s,
                       rte::launch_update(plan, C, C + 1, upd == RTE_UPDATE_SART ? rte::kUpdSartOS : rte::kUpdMlemOS,
                                          params->lambda, params->clamp_nonneg, nullptr, nullptr, 0, 0, s, nullptr,
                                          inside, plan->d_cols));
        } else {
            RTE_LAUNCH(plan, RTE_KERNEL_GATHER, s,
                       rte::launch_gather(plan, C, gmode, plan->d_y, params->alpha_l, params->alpha_d, params->tau, s,
                                          nullptr, params->g_sigma, params->seed, it));
            RTE_LAUNCH(plan, RTE_KERNEL_UPDATE, s,
                       rte::launch_update(plan, C, C, umode, params->lambda, params->clamp_nonneg, nullptr,
                                          nullptr, 0, 0, s, nullptr, inside));
        }
        plan->last_iters = it + 1;
    }
    RTE_LAUNCH(plan, RTE_KERNEL_PACK, s, rte::launch_unpack(plan, emission, C, s));
    return ok();
}

int rte_reconstruct_stats(const rte_plan *plan, int32_t *iters_done, int32_t *n_errors, float *errors,
                          int32_t max_errors)
{
    if (int rc = check_plan(plan)) return rc;
    if (iters_done) *iters_done = plan->last_iters;
    if (n_errors) *n_errors = (int32_t)plan->last_errors.size();
    if (errors)
        for (int i = 0; i < max_errors && i < (int)plan->last_errors.size(); ++i) errors[i] = plan->last_errors[i];
    return ok();
}

int rte_flame_mask(rte_plan *plan, const float *frames, float threshold, float *mask, void *stream)
{
    if (int rc = check_plan(plan)) return rc;
    if (!frames || !mask) return fail(RTE_ERR_INVALID_ARG, "null frames or mask");
    hipStream_t s = static_cast<hipStream_t>(stream);
    plan->last_stream = s;
    RTE_LAUNCH(plan, RTE_KERNEL_PACK, s, rte::launch_flame_mask(plan, frames, plan->params.channels, threshold, mask, s));
    return ok();
}

int rte_visual_hull(rte_plan *plan, const float *mask, int32_t *inside, void *stream)
{
    if (int rc = check_plan(plan)) return rc;
    if (!inside) return fail(RTE_ERR_INVALID_ARG, "null output");
    if (plan->V > 64) return fail(RTE_ERR_UNSUPPORTED, "the visual hull supports at most 64 views");
    hipStream_t s = static_cast<hipStream_t>(stream);
    plan->last_stream = s;
    RTE_LAUNCH(plan, RTE_KERNEL_GATHER, s, rte::launch_hull(plan, mask, inside, s));
    return ok();
}

int rte_job_begin(rte_plan *plan, const float *frames, const float *extinction, const float *emission,
                  const rte_recon_params *params, void *stream)
{
    if (int rc = check_plan(plan)) return rc;
    if (!frames || !extinction || !params) return fail(RTE_ERR_INVALID_ARG, "null frames, extinction or params");
    if (plan->job_open) return fail(RTE_ERR_INVALID_ARG, "the plan already has an open job");
    const int upd = params->update;
    if (upd != RTE_UPDATE_SART && upd != RTE_UPDATE_PAPER && upd != RTE_UPDATE_MLEM)
        return fail(RTE_ERR_INVALID_ARG, "unknown update rule %d", upd);
    if (!std::isfinite(params->lambda) || !(params->g_sigma >= 0.0f))
        return fail(RTE_ERR_INVALID_ARG, "lambda must be finite and g_sigma >= 0");
    if (upd == RTE_UPDATE_PAPER && !(params->tau >= 0.0f && params->tau < 1.0f))
        return fail(RTE_ERR_INVALID_ARG, "tau must be in [0, 1)");
    if (params->stop_tol != 0.0f) return fail(RTE_ERR_UNSUPPORTED, "jobs run a fixed number of steps (stop_tol = 0)");
    if (params->ordered_subsets > 1) return fail(RTE_ERR_UNSUPPORTED, "jobs update with all views at once (ordered_subsets <= 1)");
    if (params->use_hull && plan->V > 64) return fail(RTE_ERR_UNSUPPORTED, "the visual hull supports at most 64 views");
    hipStream_t s = static_cast<hipStream_t>(stream);
    plan->last_stream = s;
    const int C = plan->params.channels;
    const float *mask = params->use_mask ? plan->d_mask : nullptr;
    // emission == NULL: warm start from the volume resident in the plan
    RTE_LAUNCH(plan, RTE_KERNEL_PACK, s, rte::launch_pack(plan, emission, extinction, C, s, emission == nullptr));
    if (params->use_mask)
        RTE_LAUNCH(plan, RTE_KERNEL_PACK, s,
                   rte::launch_flame_mask(plan, frames, C, params->flame_threshold, plan->d_mask, s));
    if (params->use_hull) {
        RTE_LAUNCH(plan, RTE_KERNEL_GATHER, s, rte::launch_hull(plan, mask, plan->d_inside, s));
        RTE_LAUNCH(plan, RTE_KERNEL_UPDATE, s,
                   rte::launch_apply_outside(plan, C, plan->d_inside, params->outside_value, s));
    }
    // SART and EM: the per-sample weights and the column sums come out of
    // the job's first step (see rte_job_step)
    plan->job_open = true;
    plan->job_frames = frames;
    plan->job_params = *params;
    plan->job_iter = 0;
    return ok();
}

int rte_job_step(rte_plan *const *plans, int32_t n, void *stream)
{
    if (!plans || n < 1) return fail(RTE_ERR_INVALID_ARG, "need at least one plan");
    if (n > kMaxBatch) return fail(RTE_ERR_UNSUPPORTED, "at most %d plans per step", kMaxBatch);
    const rte_plan *p0 = plans[0];
    for (int i = 0; i < n; ++i) {
        const rte_plan *p = plans[i];
        if (!p || !p->job_open) return fail(RTE_ERR_INVALID_ARG, "plan %d has no open job", i);
        for (int k = 0; k < i; ++k)
            if (plans[k] == p) return fail(RTE_ERR_INVALID_ARG, "plan %d appears twice", i);
        if (p->params.channels != p0->params.channels || p->job_params.update != p0->job_params.update ||
            (p->params.albedo > 0.0f) != (p0->params.albedo > 0.0f))
            return fail(RTE_ERR_UNSUPPORTED, "a step batches plans with one channel count, update rule and scattering setting");
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    const bool scat = p0->params.albedo > 0.0f && p0->params.scatter_res >= 2;
    // every plan's in-scatter grid, one launch per pass for all of them
    // (timing charged to the first listed plan)
    if (scat) RTE_LAUNCH(plans[0], RTE_KERNEL_INSCATTER, s, rte::launch_inscatter_batch(plans, n, s));
    // the first step of a SART or EM job runs alone, as the first iteration
    // of rte_reconstruct does: its render also stores the per-sample weights
    // and its gather also accumulates the column sums that the later steps
    // read (so every job's steps give bitwise the rte_reconstruct result)
    rte_plan *rest[kMaxBatch];
    int nrest = 0;
    for (int i = 0; i < n; ++i) {
        rte_plan *p = plans[i];
        const rte_recon_params &q = p->job_params;
        if (p->job_iter > 0 || q.update == RTE_UPDATE_PAPER) {
            rest[nrest++] = p;
            continue;
        }
        const int C = p->params.channels;
        const float *mask = q.use_mask ? p->d_mask : nullptr;
        const bool sart = q.update == RTE_UPDATE_SART;
        RTE_LAUNCH(p, RTE_KERNEL_RENDER, s,
                   rte::launch_render(p, C, true, scat, true, sart ? rte::kEpiSart : rte::kEpiMlem, p->job_frames, C,
                                      0, p->d_y, s, nullptr, mask, nullptr));
        RTE_LAUNCH(p, RTE_KERNEL_GATHER, s,
                   rte::launch_gather(p, C, rte::kGatherAdjointCols, p->d_y, 0.f, 0.f, 0.f, s, mask));
        RTE_LAUNCH(p, RTE_KERNEL_UPDATE, s,
                   rte::launch_update(p, C, C + 1, sart ? rte::kUpdSartOS : rte::kUpdMlemOS, q.lambda, q.clamp_nonneg,
                                      nullptr, nullptr, 0, 0, s, nullptr, q.use_hull ? p->d_inside : nullptr,
                                      p->d_cols));
    }
    if (nrest == 0) {
        for (int i = 0; i < n; ++i) {
            plans[i]->job_iter += 1;
            plans[i]->last_stream = s;
        }
        return ok();
    }
    // timing of the batched launches is charged to the first plan of the batch
    rte_plan *p0t = rest[0];
    hipEvent_t marks[6] = {};
    const int kid[3] = {RTE_KERNEL_RENDER, RTE_KERNEL_GATHER, RTE_KERNEL_UPDATE};
    for (int k = 0; k < 3; ++k)
        if ((p0t->timing_mask >> kid[k]) & 1u) {
            marks[2 * k] = take_event(p0t);
            marks[2 * k + 1] = take_event(p0t);
        }
    hipError_t e = rte::launch_step_batch(rest, nrest, s, p0t->timing_mask ? marks : nullptr);
    if (p0t->timing_mask) {
        for (int k = 0; k < 3; ++k) {
            if (marks[2 * k] && marks[2 * k + 1]) {
                p0t->pending.push_back({kid[k], marks[2 * k], marks[2 * k + 1]});
            } else {
                if (marks[2 * k]) p0t->event_pool.push_back(marks[2 * k]);
                if (marks[2 * k + 1]) p0t->event_pool.push_back(marks[2 * k + 1]);
            }
        }
    }
    if (e != hipSuccess) return fail(RTE_ERR_HIP, "batched step failed: %s", hipGetErrorString(e));
    for (int i = 0; i < n; ++i) {
        plans[i]->job_iter += 1;
        plans[i]->last_stream = s;
    }
    return ok();
}

int rte_job_end(rte_plan *plan, float *emission, void *stream)
{
    if (int rc = check_plan(plan)) return rc;
    if (!plan->job_open) return fail(RTE_ERR_INVALID_ARG, "the plan has no open job");
    hipStream_t s = static_cast<hipStream_t>(stream);
    plan->last_stream = s;
    if (emission) RTE_LAUNCH(plan, RTE_KERNEL_PACK, s, rte::launch_unpack(plan, emission, plan->params.channels, s));
    plan->last_iters = plan->job_iter;
    plan->job_open = false;
    plan->job_frames = nullptr;
    return ok();
}

int rte_reconstruct_temperature(rte_plan *plan, const float *frames, float *temperature, int32_t iters,
                                const rte_recon_params *params, const rte_temp_params *temp, void *stream)
{
    if (int rc = check_plan(plan)) return rc;
    if (!frames || !temperature || !params || !temp)
        return fail(RTE_ERR_INVALID_ARG, "null frames, temperature or params");
    if (plan->params.channels != 1) return fail(RTE_ERR_INVALID_ARG, "temperature fit needs a plan with channels = 1");
    if (iters < 0) return fail(RTE_ERR_INVALID_ARG, "iters must be >= 0");
    if (!std::isfinite(params->lambda)) return fail(RTE_ERR_INVALID_ARG, "lambda must be finite");
    hipStream_t s = static_cast<hipStream_t>(stream);
    plan->last_stream = s;
    if (int rc = ensure_lut(plan, temp, s)) return rc;
    const rte_temp_params &tp = *temp;
    for (int it = 0; it < iters; ++it) {
        RTE_LAUNCH(plan, RTE_KERNEL_TEMP_MAP, s,
                   rte::launch_temp_map(plan, temperature, nullptr, nullptr, true, tp.lut_size, tp.channel,
                                        tp.sigma_max, tp.soot_t0, tp.soot_span, tp.t_min, tp.t_max, s));
        RTE_LAUNCH(plan, RTE_KERNEL_RENDER, s,
                   rte::launch_render(plan, 1, true, false, true, rte::kEpiMlem, frames, 3, tp.channel, plan->d_y, s));
        RTE_LAUNCH(plan, RTE_KERNEL_GATHER, s,
                   rte::launch_gather(plan, 1, rte::kGatherAdjointCols, plan->d_y, 0.f, 0.f, 0.f, s));
        RTE_LAUNCH(plan, RTE_KERNEL_UPDATE, s,
                   rte::launch_update(plan, 1, 2, rte::kUpdTemp, params->lambda, 0, nullptr, temperature,
                                      tp.lut_size, tp.channel, s));
    }
    return ok();
}

int rte_temperature_map(rte_plan *plan, const float *temperature, float *emission, float *extinction,
                        const rte_temp_params *temp, void *stream)
{
    if (int rc = check_plan(plan)) return rc;
    if (!temperature || (!emission && !extinction)) return fail(RTE_ERR_INVALID_ARG, "null temperature or no output");
    hipStream_t s = static_cast<hipStream_t>(stream);
    plan->last_stream = s;
    if (int rc = ensure_lut(plan, temp, s)) return rc;
    RTE_LAUNCH(plan, RTE_KERNEL_TEMP_MAP, s,
               rte::launch_temp_map(plan, temperature, emission, extinction, false, temp->lut_size, temp->channel,
                                    temp->sigma_max, temp->soot_t0, temp->soot_span, temp->t_min, temp->t_max, s));
    return ok();
}

int rte_temperature_invert(rte_plan *plan, const float *e, float *temperature, const rte_temp_params *temp,
                           void *stream)
{
    if (int rc = check_plan(plan)) return rc;
    if (!e || !temperature) return fail(RTE_ERR_INVALID_ARG, "null input or output");
    hipStream_t s = static_cast<hipStream_t>(stream);
    plan->last_stream = s;
    if (int rc = ensure_lut(plan, temp, s)) return rc;
    RTE_LAUNCH(plan, RTE_KERNEL_TEMP_MAP, s,
               rte::launch_temp_invert(plan, e, temperature, temp->lut_size, temp->channel, temp->t_min,
                                       temp->t_max, s));
    return ok();
}

int rte_temperature_lut(rte_plan *plan, const rte_temp_params *temp, float *lut_host, int32_t lut_size)
{
    if (int rc = check_plan(plan)) return rc;
    if (!temp || !lut_host || lut_size != temp->lut_size)
        return fail(RTE_ERR_INVALID_ARG, "null arguments or lut_size mismatch");
    if (int rc = ensure_lut(plan, temp, plan->last_stream)) return rc;
    std::memcpy(lut_host, plan->lut_host.data(), sizeof(float) * 3 * (size_t)lut_size);
    return ok();
}

int rte_plan_set_timing_mask(rte_plan *plan, uint32_t kernels)
{
    if (int rc = check_plan(plan)) return rc;
    if (kernels >> RTE_KERNEL_COUNT) return fail(RTE_ERR_INVALID_ARG, "timing mask 0x%x names no kernel", kernels);
    drain_timing(plan);
    plan->timing_mask = kernels;
    for (int k = 0; k < RTE_KERNEL_COUNT; ++k) {
        plan->kernel_ms[k] = 0.0;
        plan->kernel_launches[k] = 0;
    }
    if (plan->timing_mask && plan->event_pool.empty()) {
        for (int i = 0; i < 256; ++i) {
            hipEvent_t e = make_timing_event();
            if (!e) return fail(RTE_ERR_HIP, "hipEventCreateWithFlags failed");
            plan->event_pool.push_back(e);
        }
    }
    return ok();
}

int rte_plan_set_timing(rte_plan *plan, int32_t enable)
{
    return rte_plan_set_timing_mask(plan, enable ? (1u << RTE_KERNEL_COUNT) - 1u : 0u);
}

int rte_plan_kernel_time(rte_plan *plan, int32_t kernel, double *total_ms, int64_t *launches)
{
    if (int rc = check_plan(plan)) return rc;
    if (kernel < 0 || kernel >= RTE_KERNEL_COUNT) return fail(RTE_ERR_INVALID_ARG, "unknown kernel id %d", kernel);
    drain_timing(plan);
    if (total_ms) *total_ms = plan->kernel_ms[kernel];
    if (launches) *launches = plan->kernel_launches[kernel];
    return ok();
}

}  // extern "C"
