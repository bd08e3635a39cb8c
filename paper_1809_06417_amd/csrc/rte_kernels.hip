// HIP kernels of librte for gfx950 (MI355X, CDNA4, wave64).
//
// K4 ray table   : once per plan, FP64 ray/box geometry per pixel ray.
// K1 render      : one work-item per pixel ray, one wave per 8x8 pixel tile,
//                  front-to-back march (Eq. 5-8) with fused residual epilogue
//                  and optional per-sample weight output.
// K2 in-scatter  : direction-major march from every in-scatter node (a wave
//                  per 4x4x4 node brick, directions spread over the XCDs),
//                  then a fixed-order sum over directions (Eq. 5 third
//                  term, Eq. 9 at g = 0).
// K3 gather      : atomics-free back-projection (Alg. 2 adjustment): each
//                  work-item owns one voxel (cell) and gathers, per view, the
//                  samples of the rays through that cell into per-corner
//                  partial sums; an assembly pass sums the eight cells around
//                  every key point in a fixed order and applies the update.
// K5 temperature : LUT map T -> (eps, sigma) and its inverse (Eq. 13).
//
// No float atomics anywhere: every sum has a fixed order, so results are
// bitwise reproducible run to run.
#include <climits>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "rte_internal.h"

namespace rte {
namespace {

constexpr int kBlock = 256;

// ------------------------------------------------------------------ helpers

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2). Give XCD x a contiguous range of logical blocks so that neighbouring
// tiles / bricks share an L2. nb8 is the launched grid (a multiple of 8).
__device__ __forceinline__ int xcd_remap(int b, int nb8)
{
    const int per = nb8 >> 3;
    return (b & 7) * per + (b >> 3);
}

static inline int grid8(int64_t blocks) { return (int)(((blocks + 7) / 8) * 8); }

// Segment k of a chord of length L marched with step ds: midpoint offset s
// from the entry and length len; the last segment is clipped at the exit.
__device__ __forceinline__ void segment_of(int k, int K, float L, float ds, float &s, float &len)
{
    // both forms are evaluated and one is selected (no branch in the march loops)
    const float a = (float)k * ds;
    const float len_last = __builtin_amdgcn_fmed3f(L - a, 0.0f, ds);
    const bool inner = k < K - 1;
    len = inner ? ds : len_last;
    s = inner ? ((float)k + 0.5f) * ds : fmaf(0.5f, len_last, a);
}

// Clamp a grid coordinate to [0, n-1] and split it into a cell index
// (<= n-2) and the fraction inside the cell.
__device__ __forceinline__ void cell_of(float x, int n, int &i, float &f)
{
    x = __builtin_amdgcn_fmed3f(x, 0.0f, (float)(n - 1));
    i = min((int)x, n - 2);
    f = x - (float)i;
}

// Trilinear weights of the 8 cell corners, corner index = dx + 2 dy + 4 dz.
__device__ __forceinline__ void tri_weights(float fx, float fy, float fz, float w[8])
{
    const float ax0 = 1.0f - fx, ay0 = 1.0f - fy, az0 = 1.0f - fz;
    const float b00 = ay0 * az0, b10 = fy * az0, b01 = ay0 * fz, b11 = fy * fz;
    w[0] = ax0 * b00;
    w[1] = fx * b00;
    w[2] = ax0 * b10;
    w[3] = fx * b10;
    w[4] = ax0 * b01;
    w[5] = fx * b01;
    w[6] = ax0 * b11;
    w[7] = fx * b11;
}

// phi(x) = (1 - e^-x) / x (segment-averaged transmittance) and e = e^-x.
// Taylor series below x = 0.25 (truncation < 2e-9), direct form above.
__device__ __forceinline__ float phi_exp(float x, float &e)
{
    e = __expf(-x);
    const float ser =
        fmaf(x, fmaf(x, fmaf(x, fmaf(x, fmaf(x, fmaf(x, 1.0f / 5040.0f, -1.0f / 720.0f), 1.0f / 120.0f),
                                          -1.0f / 24.0f),
                             1.0f / 6.0f),
                  -0.5f),
             1.0f);
    const float dir = (1.0f - e) * __builtin_amdgcn_rcpf(x);
    return x < 0.25f ? ser : dir;
}

// Raw buffer resource over [p, p + bytes): loads take a 32-bit lane offset
// plus a uniform (SGPR) offset, and the hardware returns 0 for any access
// outside the range instead of touching other memory.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *p, int64_t bytes)
{
    const int n = bytes > 0x7fffffff ? 0x7fffffff : (int)bytes;
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, n, 0x00020000);
}

__device__ __forceinline__ float4 bload4(__amdgpu_buffer_rsrc_t r, int voff, int soff)
{
    using u4 = unsigned int __attribute__((ext_vector_type(4)));
    const u4 v = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
    return make_float4(__uint_as_float(v.x), __uint_as_float(v.y), __uint_as_float(v.z),
                       __uint_as_float(v.w));
}

__device__ __forceinline__ float2 bload2(__amdgpu_buffer_rsrc_t r, int voff, int soff)
{
    using u2 = unsigned int __attribute__((ext_vector_type(2)));
    const u2 v = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
    return make_float2(__uint_as_float(v.x), __uint_as_float(v.y));
}

template <int C> struct Packed;
template <> struct Packed<1> { using T = float2; };
template <> struct Packed<3> { using T = float4; };

// Trilinear sample of a packed volume through a buffer resource: coff holds
// the byte offsets of the 8 cell corners (uniform across the launch). The
// corners of the last cell sampled are kept (a march at half a voxel per step
// stays in one cell for about every other sample): they are reloaded only
// when the cell changes, and the interpolation is the same as with a fresh
// load.
template <int C>
struct VolCorners {
    using T = typename Packed<C>::T;
    int cell = -1;
    T v[8];
};

// Trilinear interpolation of the 8 corner values, corners in index order
// (every sampler of the packed volume uses these products in this order).
template <int C>
__device__ __forceinline__ void interp_corners(const typename Packed<C>::T v[8], const float w[8], float em[C],
                                               float &sig)
{
    sig = 0.0f;
#pragma unroll
    for (int c = 0; c < C; ++c) em[c] = 0.0f;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        if constexpr (C == 3) {
            em[0] = fmaf(w[c], v[c].x, em[0]);
            em[1] = fmaf(w[c], v[c].y, em[1]);
            em[2] = fmaf(w[c], v[c].z, em[2]);
            sig = fmaf(w[c], v[c].w, sig);
        } else {
            em[0] = fmaf(w[c], v[c].x, em[0]);
            sig = fmaf(w[c], v[c].y, sig);
        }
    }
}

template <int C>
__device__ __forceinline__ void sample_volume_rsrc(__amdgpu_buffer_rsrc_t r, const int coff[8], int base_bytes,
                                                   const float w[8], VolCorners<C> &vc, float em[C], float &sig)
{
    if (base_bytes != vc.cell) {
        vc.cell = base_bytes;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            if constexpr (C == 3) vc.v[c] = bload4(r, base_bytes, coff[c]);
            else vc.v[c] = bload2(r, base_bytes, coff[c]);
        }
    }
    interp_corners<C>(vc.v, w, em, sig);
}

__device__ __forceinline__ void corner_offsets(int nx, int nxy, int elem, int coff[8])
{
#pragma unroll
    for (int c = 0; c < 8; ++c)
        coff[c] = ((c & 1) + ((c >> 1) & 1) * nx + ((c >> 2) & 1) * nxy) * elem;
}

// Philox-4x32-10 counter-based generator (Salmon et al., SC 2011).
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = 0xD2511F53u * c[0], hi0 = __umulhi(0xD2511F53u, c[0]);
        const uint32_t lo1 = 0xCD9E8D57u * c[2], hi1 = __umulhi(0xCD9E8D57u, c[2]);
        const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// Per-sample gain G(s) of Eq. 11: 1 + g_sigma * z, z standard normal by
// Box-Muller from two Philox words keyed by the seed, counter (k, pixel,
// view, iteration).
__device__ __forceinline__ float sample_gain(uint32_t seed_lo, uint32_t seed_hi, int it, int v, int pix, int k,
                                             float g_sigma)
{
    uint32_t c[4] = {(uint32_t)k, (uint32_t)pix, (uint32_t)v, (uint32_t)it};
    philox4x32_10(c, seed_lo, seed_hi);
    const float u1 = ((float)(c[0] >> 8) + 0.5f) * (1.0f / 16777216.0f);
    const float u2 = ((float)(c[1] >> 8) + 0.5f) * (1.0f / 16777216.0f);
    const float z = sqrtf(-2.0f * logf(u1)) * cosf(6.283185307179586f * u2);
    return fmaf(g_sigma, z, 1.0f);
}


// ------------------------------------------------------------- K4 ray table

struct RayArgs {
    const rte_camera *cams;
    float4 *rayA, *rayB;
    float *tnear;
    int W, H, V;
    double lo[3], hi[3], h[3];
    double ds;
};

// FP64 geometry: pinhole direction R^T K^-1 (u+1/2, v+1/2, 1), slab entry and
// exit, K = ceil(chord / step). Contraction is off so the integer segment
// count is decided by correctly rounded IEEE operations.
__global__ __launch_bounds__(kBlock) void ray_table_kernel(RayArgs a)
{
#pragma clang fp contract(off)
    const int64_t HW = (int64_t)a.W * a.H;
    const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (r >= HW * a.V) return;
    const int v = (int)(r / HW);
    const int64_t pix = r - (int64_t)v * HW;
    const int py = (int)(pix / a.W), px = (int)(pix - (int64_t)py * a.W);
    const rte_camera &c = a.cams[v];
    const double dc0 = ((double)px + 0.5 - c.cx) / c.fx;
    const double dc1 = ((double)py + 0.5 - c.cy) / c.fy;
    const double dc2 = 1.0;
    double d[3], o[3], n2 = 0.0;
    for (int i = 0; i < 3; ++i) {
        d[i] = c.R[0 * 3 + i] * dc0 + c.R[1 * 3 + i] * dc1 + c.R[2 * 3 + i] * dc2;
        o[i] = -(c.R[0 * 3 + i] * c.t[0] + c.R[1 * 3 + i] * c.t[1] + c.R[2 * 3 + i] * c.t[2]);
        n2 += d[i] * d[i];
    }
    const double inv = 1.0 / sqrt(n2);
    for (int i = 0; i < 3; ++i) d[i] *= inv;
    double t0 = -INFINITY, t1 = INFINITY;
    bool hit = true;
    for (int i = 0; i < 3; ++i) {
        if (d[i] != 0.0) {
            double ta = (a.lo[i] - o[i]) / d[i], tb = (a.hi[i] - o[i]) / d[i];
            if (ta > tb) {
                const double s = ta;
                ta = tb;
                tb = s;
            }
            if (ta > t0) t0 = ta;
            if (tb < t1) t1 = tb;
        } else if (o[i] < a.lo[i] || o[i] > a.hi[i]) {
            hit = false;
        }
    }
    if (t0 < 0.0) t0 = 0.0;
    hit = hit && (t1 > t0);
    int K = 0;
    float4 A = make_float4(0.f, 0.f, 0.f, 0.f), B = make_float4(0.f, 0.f, 0.f, 0.f);
    if (hit) {
        K = (int)ceil((t1 - t0) / a.ds);
        double p[3];
        for (int i = 0; i < 3; ++i) p[i] = (o[i] + t0 * d[i] - a.lo[i]) / a.h[i];
        A = make_float4((float)p[0], (float)p[1], (float)p[2], (float)(t1 - t0));
        B = make_float4((float)(d[0] / a.h[0]), (float)(d[1] / a.h[1]), (float)(d[2] / a.h[2]), 0.f);
    }
    B.w = __int_as_float(K);
    a.rayA[r] = A;
    a.rayB[r] = B;
    a.tnear[r] = hit ? (float)t0 : 0.0f;
}

struct TileArgs {
    const float4 *rayB;
    int32_t *kmax;
    int W, H, tiles_x, tiles_per_view, n_tiles;
};

// Maximum segment count of every 8x8 tile (sizes the per-sample weight rows).
__global__ __launch_bounds__(kTileRays) void tile_kmax_kernel(TileArgs a)
{
    const int tile = blockIdx.x;
    if (tile >= a.n_tiles) return;
    const int lane = threadIdx.x;
    const int v = tile / a.tiles_per_view, t = tile - v * a.tiles_per_view;
    const int ty = t / a.tiles_x, tx = t - ty * a.tiles_x;
    const int px = tx * kTile + (lane & 7), py = ty * kTile + (lane >> 3);
    int K = 0;
    if (px < a.W && py < a.H)
        K = __float_as_int(a.rayB[((int64_t)v * a.H + py) * a.W + px].w);
    for (int off = 32; off > 0; off >>= 1) K = max(K, __shfl_xor(K, off, 64));
    if (lane == 0) a.kmax[tile] = K;
}

struct ExportArgs {
    const float4 *rayA, *rayB;
    const float *tnear;
    float *t_near, *t_far;
    int32_t *nseg;
    int64_t n;
};

__global__ __launch_bounds__(kBlock) void ray_export_kernel(ExportArgs a)
{
    const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (r >= a.n) return;
    const int K = __float_as_int(a.rayB[r].w);
    const float tn = a.tnear[r];
    if (a.t_near) a.t_near[r] = tn;
    if (a.t_far) a.t_far[r] = K > 0 ? tn + a.rayA[r].w : 0.0f;
    if (a.nseg) a.nseg[r] = K;
}

// ----------------------------------------------------------------- packing

struct PackArgs {
    const float *em, *sig;
    float *vol;
    int64_t n;
    int keep_emission;  // 1: only the extinction slot is written (warm start)
};

template <int C>
__global__ __launch_bounds__(kBlock) void pack_kernel(PackArgs a)
{
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= a.n) return;
    const float s = a.sig ? a.sig[j] : 0.0f;
    if (a.keep_emission) {
        if constexpr (C == 3) reinterpret_cast<float4 *>(a.vol)[j].w = s;
        else reinterpret_cast<float2 *>(a.vol)[j].y = s;
        return;
    }
    if constexpr (C == 3) {
        float4 v = make_float4(0.f, 0.f, 0.f, s);
        if (a.em) {
            v.x = a.em[j];
            v.y = a.em[a.n + j];
            v.z = a.em[2 * a.n + j];
        }
        reinterpret_cast<float4 *>(a.vol)[j] = v;
    } else {
        reinterpret_cast<float2 *>(a.vol)[j] = make_float2(a.em ? a.em[j] : 0.0f, s);
    }
}

template <int C>
__global__ __launch_bounds__(kBlock) void unpack_kernel(PackArgs a, float *em)
{
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= a.n) return;
    if constexpr (C == 3) {
        const float4 v = reinterpret_cast<const float4 *>(a.vol)[j];
        em[j] = v.x;
        em[a.n + j] = v.y;
        em[2 * a.n + j] = v.z;
    } else {
        em[j] = reinterpret_cast<const float2 *>(a.vol)[j].x;
    }
}

__global__ __launch_bounds__(kBlock) void pack_scatter_kernel(const float *planar, float4 *out, int C,
                                                             int64_t m3)
{
    const int64_t m = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (m >= m3) return;
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    v.x = planar[m];
    if (C == 3) {
        v.y = planar[m3 + m];
        v.z = planar[2 * m3 + m];
    }
    out[m] = v;
}

// In-scatter corners of the coarse cell a ray is in. The coarse grid is
// several fine cells wide, so consecutive samples mostly stay in one coarse
// cell: the eight corners are reloaded only when the cell changes (the
// values and the interpolation order are those of a fresh load).
struct ScatCorners {
    int cell = -1;
    float v[8][3];
};

__device__ __forceinline__ void scat_sample(const __amdgpu_buffer_rsrc_t &sr, const int soff[8], int sb,
                                            const float ws[8], ScatCorners &cc, float S[3])
{
    if (sb != cc.cell) {
        cc.cell = sb;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const float4 q = bload4(sr, sb, soff[c]);
            cc.v[c][0] = q.x;
            cc.v[c][1] = q.y;
            cc.v[c][2] = q.z;
        }
    }
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        S[0] = fmaf(ws[c], cc.v[c][0], S[0]);
        S[1] = fmaf(ws[c], cc.v[c][1], S[1]);
        S[2] = fmaf(ws[c], cc.v[c][2], S[2]);
    }
}

// LDS window of the packed volume for the rays of one wave (an 8x8 pixel
// tile). The tile's rays stay close together, so at each step their samples
// fall in a few cells: the wave keeps an 8x8x8-node window in LDS, addressed
// toroidally (node (x, y, z) in the slot of (x & 7, y & 7, z & 7)), and reads the 8
// corners of every sample from it. When a sample leaves the window, the wave
// moves the window so that it starts at the rays' trailing cells along the
// march direction and loads only the node planes that enter it (one
// coalesced plane of 64 nodes per load instruction). A sample the window
// cannot hold (the rays spread over more than 6 cells) reads its corners
// from memory. The corner values are the same either way.
constexpr int kWin = 8;

// Slot of node (x, y, z) (coordinates mod 8): x + 9 y + 72 z, rows padded to
// 9 slots. The LDS banks serve a 16-byte node per 4 banks, so the slot mod 16
// picks the bank group; with the padding, nodes one apart along x, y or the
// xy diagonal fall in different groups, and the rays of a pixel row, which
// sit side by side across the march direction, rarely share a group (in
// plain 8 x 8 x 8 order they did 3-4 at a time). The corners of a cell are
// the slot plus fixed steps (+1, +9, +72, or -7, -63, -504 where the
// coordinate wraps from 7 to 0).
constexpr int kWinPitchY = 9, kWinPitchZ = 72;
constexpr int kWinSlots = 576;
__device__ __forceinline__ int win_slot(int x, int y, int z)
{
    return (x & 7) + kWinPitchY * (y & 7) + kWinPitchZ * (z & 7);
}

template <int C>
__device__ __forceinline__ typename Packed<C>::T vload(__amdgpu_buffer_rsrc_t r, int off)
{
    if constexpr (C == 3) return bload4(r, off, 0);
    else return bload2(r, off, 0);
}

// Load the planes p in [p0, p1) normal to axis `ax` of the window whose other
// two axes start at (o1, o2); lane l takes node (l & 7, l >> 3) of a plane.
template <int C>
__device__ __forceinline__ void win_planes(typename Packed<C>::T *lds, __amdgpu_buffer_rsrc_t vr, int ax, int p0,
                                           int p1, int o1, int o2, int nx, int ny, int nz, int lane)
{
    constexpr int elem = C == 3 ? 16 : 8;
    const int a1 = lane & 7, a2 = lane >> 3;
    for (int q = p0; q < p1; ++q) {
        const int x = ax == 0 ? q : o1 + a1;
        const int y = ax == 1 ? q : (ax == 0 ? o1 + a1 : o2 + a2);
        const int z = ax == 2 ? q : o2 + a2;
        if (x >= 0 && x < nx && y >= 0 && y < ny && z >= 0 && z < nz)
            lds[win_slot(x, y, z)] = vload<C>(vr, ((z * ny + y) * nx + x) * elem);
    }
}

__device__ __forceinline__ int wave_min(int v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
    return v;
}

__device__ __forceinline__ int wave_max(int v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
    return v;
}

// Window origin for one axis: the trailing cell of the wave's samples along
// the march direction, kept inside the grid.
__device__ __forceinline__ int win_origin(int mn, int mx, bool forward, int n)
{
    int o = forward ? mn : mx - (kWin - 2);
    o = min(o, n - kWin);
    return max(o, 0);
}

template <int C>
struct VolWindow {
    typename Packed<C>::T *lds;
    int ox = 0, oy = 0, oz = 0;
    bool valid = false;
    bool fx = true, fy = true, fz = true;  // march direction sign per axis

    // All lanes of the wave call this with their sample's cell; returns
    // whether the lane's 8 corners are in the window afterwards.
    __device__ __forceinline__ bool update(bool act, int ix, int iy, int iz, __amdgpu_buffer_rsrc_t vr, int nx,
                                           int ny, int nz, int lane)
    {
        auto inside = [&](int x0, int y0, int z0) {
            return (unsigned)(ix - x0) <= (unsigned)(kWin - 2) && (unsigned)(iy - y0) <= (unsigned)(kWin - 2) &&
                   (unsigned)(iz - z0) <= (unsigned)(kWin - 2);
        };
        const bool need = act && !(valid && inside(ox, oy, oz));
        if (__ballot(need) == 0) return act;
        const int mnx = wave_min(act ? ix : INT_MAX), mxx = wave_max(act ? ix : INT_MIN);
        const int mny = wave_min(act ? iy : INT_MAX), mxy = wave_max(act ? iy : INT_MIN);
        const int mnz = wave_min(act ? iz : INT_MAX), mxz = wave_max(act ? iz : INT_MIN);
        const int nox = __builtin_amdgcn_readfirstlane(win_origin(mnx, mxx, fx, nx));
        const int noy = __builtin_amdgcn_readfirstlane(win_origin(mny, mxy, fy, ny));
        const int noz = __builtin_amdgcn_readfirstlane(win_origin(mnz, mxz, fz, nz));
        const int dx = nox - ox, dy = noy - oy, dz = noz - oz;
        if (!valid || abs(dx) >= kWin || abs(dy) >= kWin || abs(dz) >= kWin) {
            win_planes<C>(lds, vr, 2, noz, noz + kWin, nox, noy, nx, ny, nz, lane);
        } else {
            // planes entering the window along each axis (edges may load twice)
            if (dx > 0) win_planes<C>(lds, vr, 0, ox + kWin, nox + kWin, noy, noz, nx, ny, nz, lane);
            if (dx < 0) win_planes<C>(lds, vr, 0, nox, ox, noy, noz, nx, ny, nz, lane);
            if (dy > 0) win_planes<C>(lds, vr, 1, oy + kWin, noy + kWin, nox, noz, nx, ny, nz, lane);
            if (dy < 0) win_planes<C>(lds, vr, 1, noy, oy, nox, noz, nx, ny, nz, lane);
            if (dz > 0) win_planes<C>(lds, vr, 2, oz + kWin, noz + kWin, nox, noy, nx, ny, nz, lane);
            if (dz < 0) win_planes<C>(lds, vr, 2, noz, oz, nox, noy, nx, ny, nz, lane);
        }
        ox = nox;
        oy = noy;
        oz = noz;
        valid = true;
        return act && inside(ox, oy, oz);
    }

    // Trilinear sample from the window (same products and order as
    // sample_volume_rsrc).
    __device__ __forceinline__ void sample(int ix, int iy, int iz, const float w[8], float em[C], float &sig) const
    {
        sig = 0.0f;
#pragma unroll
        for (int c = 0; c < C; ++c) em[c] = 0.0f;
        const int xm = ix & 7, ym = iy & 7, zm = iz & 7;
        const int b0 = xm + kWinPitchY * ym + kWinPitchZ * zm;
        const int ox = xm == 7 ? -7 : 1;
        const int oy = ym == 7 ? -7 * kWinPitchY : kWinPitchY;
        const int oz = zm == 7 ? -7 * kWinPitchZ : kWinPitchZ;
        const int sl[8] = {b0, b0 + ox, b0 + oy, b0 + oy + ox, b0 + oz, b0 + oz + ox, b0 + oz + oy, b0 + oz + oy + ox};
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const auto v = lds[sl[c]];
            if constexpr (C == 3) {
                em[0] = fmaf(w[c], v.x, em[0]);
                em[1] = fmaf(w[c], v.y, em[1]);
                em[2] = fmaf(w[c], v.z, em[2]);
                sig = fmaf(w[c], v.w, sig);
            } else {
                em[0] = fmaf(w[c], v.x, em[0]);
                sig = fmaf(w[c], v.y, sig);
            }
        }
    }
};

// ---------------------------------------------------------------- K1 render

struct RenderArgs {
    const float4 *rayA, *rayB;
    const uint32_t *tile_off;  // first slot of each tile in the per-sample buffers
    const int32_t *tile_order;  // tiles with samples (heaviest first), then empty tiles
    int n_launch;               // leading entries of tile_order this launch covers
    const float *vol;
    const float4 *scat;
    int scat_vstride;    // float4 entries between the grids of consecutive views (0: one grid)
    const float *frames;
    float *out;
    float *g;
    double *exit_tau;  // optional [V][H][W] optical depth at the exit (image renders)
    const float *mask;   // optional [V][H][W] ray mask (1 adjust, 0 ignore) for residual epilogues
    float2 *err;         // optional per-slot (sum of squared residuals, count) over masked pixels
    int sub_n, sub_s;    // only views v with v % sub_n == sub_s (ordered subsets)
    int fC, fc0;  // frames hold fC channels; channel c of the render reads fc0 + c
    int W, H, tiles_x, tiles_per_view, n_tiles, nb8;
    int nx, ny, nz, M;
    float ds, albedo, background;
    float s_scale[3];  // fine grid coords -> in-scatter grid coords
};

// One work-item per pixel ray; a block holds four 8x8 tiles (one per wave).
// Tiles are taken in plan order: tiles that some ray of the volume crosses,
// heaviest (largest segment count) first, so the long marches start early
// and the short ones fill the tail; empty tiles come last and are launched
// only when an image (background for misses) is written.
// EMIS: read the emission (false: weights only). SCAT: add in-scattering.
// WRITE_G: store the per-sample weight g_k = T_k Delta_k phi_k.
template <int C, bool EMIS, bool SCAT, bool WRITE_G, int EPI>
__device__ __forceinline__ void render_body(const RenderArgs &a, int blk)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int slot = blk * 4 + wave;
    if (slot >= a.n_launch) return;
    // every lane of the wave reads the same entry: keep the tile (and so the
    // view and the per-view in-scatter grid address) in scalar registers
    const int tile = __builtin_amdgcn_readfirstlane(a.tile_order[slot]);
    if (tile < 0) {  // an empty slot of an XCD's band
        if (a.err && lane == 0) a.err[slot] = make_float2(0.0f, 0.0f);
        return;
    }
    const int v = tile / a.tiles_per_view, t = tile - v * a.tiles_per_view;
    if (a.sub_n > 1 && v % a.sub_n != a.sub_s) return;  // whole wave: view outside the subset
    const int ty = t / a.tiles_x, tx = t - ty * a.tiles_x;
    const int px = tx * kTile + (lane & 7), py = ty * kTile + (lane >> 3);
    const bool in_image = px < a.W && py < a.H;
    // lanes past the image edge stay: they take part in the wave's window
    // loads and in the tile's error butterfly
    const int HW = a.W * a.H;
    const int pix = in_image ? py * a.W + px : 0;
    const int r = v * HW + pix;
    const float4 A = a.rayA[r], B = a.rayB[r];
    const int K = in_image ? __float_as_int(B.w) : 0;
    const int nx = a.nx, nxy = a.nx * a.ny;
    constexpr int elem = C == 3 ? 16 : 8;
    const __amdgpu_buffer_rsrc_t vr = make_rsrc(a.vol, (int64_t)nxy * a.nz * elem);
    int coff[8];
    corner_offsets(nx, nxy, elem, coff);
    const int M = a.M, MM = a.M * a.M;
    const __amdgpu_buffer_rsrc_t sr =
        make_rsrc(a.scat + (int64_t)v * a.scat_vstride, SCAT ? (int64_t)MM * M * 16 : 16);
    int soff[8];
    corner_offsets(M, MM, 16, soff);
    float I[C];
#pragma unroll
    for (int c = 0; c < C; ++c) I[c] = 0.0f;
    float T = 1.0f, Rsum = 0.0f;
    // optical depth so far, in FP64: an image render hands it to the reverse
    // march, which recovers every T_k from it even where T_K underflows
    double tau = 0.0;
    // per-sample weights: stored as 16-byte groups of four steps
    float4 *gp = nullptr;
    if constexpr (WRITE_G) gp = reinterpret_cast<float4 *>(a.g + a.tile_off[tile]) + lane;
    ScatCorners scc;
    __shared__ typename Packed<C>::T win_lds[4][kWinSlots];
    VolWindow<C> win;
    win.lds = win_lds[wave];
    {
        // march direction of the tile (sum over its rays) per axis
        float sx = B.x, sy = B.y, sz = B.z;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            sx += __shfl_xor(sx, off, 64);
            sy += __shfl_xor(sy, off, 64);
            sz += __shfl_xor(sz, off, 64);
        }
        win.fx = sx >= 0.0f;
        win.fy = sy >= 0.0f;
        win.fz = sz >= 0.0f;
    }
    // all lanes step together up to the tile's longest march
    const int Kw = wave_max(K);
    // one march step; returns the sample's weight g_k (0 past the ray's end)
    auto step = [&](int k) -> float {
        const bool act = k < K;
        float s = 0.0f, len = 0.0f;
        if (act) segment_of(k, K, A.w, a.ds, s, len);
        const float x = fmaf(s, B.x, A.x), y = fmaf(s, B.y, A.y), z = fmaf(s, B.z, A.z);
        int ix, iy, iz;
        float fx, fy, fz;
        cell_of(x, a.nx, ix, fx);
        cell_of(y, a.ny, iy, fy);
        cell_of(z, a.nz, iz, fz);
        const bool in_win = win.update(act, ix, iy, iz, vr, a.nx, a.ny, a.nz, lane);
        if (!act) return 0.0f;
        float w[8];
        tri_weights(fx, fy, fz, w);
        float em[C], sig;
        if (in_win) {
            win.sample(ix, iy, iz, w, em, sig);
        } else {
            VolCorners<C> vcc;
            const int base = (int)(__umul24(iz, nxy) + __umul24(iy, nx)) + ix;
            sample_volume_rsrc<C>(vr, coff, base * elem, w, vcc, em, sig);
        }
        sig = fmaxf(sig, 0.0f);
        if constexpr (SCAT) {
            int jx, jy, jz;
            float gx, gy, gz;
            cell_of(x * a.s_scale[0], M, jx, gx);
            cell_of(y * a.s_scale[1], M, jy, gy);
            cell_of(z * a.s_scale[2], M, jz, gz);
            float ws[8];
            tri_weights(gx, gy, gz, ws);
            const int sb = ((int)(__umul24(jz, MM) + __umul24(jy, M)) + jx) * 16;
            float S[3] = {0.f, 0.f, 0.f};
            scat_sample(sr, soff, sb, ws, scc, S);
            const float as = a.albedo * sig;
#pragma unroll
            for (int c = 0; c < C; ++c) em[c] = fmaf(as, S[c], em[c]);
        }
        float e;
        const float xo = sig * len;
        const float ph = phi_exp(xo, e);
        const float wg = T * len * ph;
        if constexpr (EPI == kEpiImage) tau += (double)xo;
        if constexpr (EMIS) {
#pragma unroll
            for (int c = 0; c < C; ++c) I[c] = fmaf(wg, em[c], I[c]);
        }
        Rsum += wg;
        T *= e;
        return wg;
    };
    if constexpr (WRITE_G) {
        // four steps per group of the weight buffer, each weight computed
        // into its place; the wave-uniform bounds keep every lane stepping
        for (int k0 = 0; k0 < Kw; k0 += kGroup) {
            float4 g4;
            g4.x = step(k0);
            g4.y = k0 + 1 < Kw ? step(k0 + 1) : 0.0f;
            g4.z = k0 + 2 < Kw ? step(k0 + 2) : 0.0f;
            g4.w = k0 + 3 < Kw ? step(k0 + 3) : 0.0f;
            if (k0 < K) gp[(k0 / kGroup) * kTileRays] = g4;
        }
    } else {
        for (int k = 0; k < Kw; ++k) step(k);
    }
    if constexpr (EPI == kEpiImage) {
        if (in_image) {
#pragma unroll
            for (int c = 0; c < C; ++c) a.out[(v * C + c) * HW + pix] = fmaf(T, a.background, I[c]);
            if (a.exit_tau) a.exit_tau[r] = tau;
        }
    } else if constexpr (EPI == kEpiSart || EPI == kEpiMlem || EPI == kEpiPaper) {
        const float m = !in_image ? 0.0f : (a.mask ? a.mask[r] : 1.0f);
        const float inv = Rsum > 0.0f ? 1.0f / Rsum : 0.0f;
        float r2 = 0.0f;
        float yo[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const float F = in_image ? a.frames[(v * a.fC + a.fc0 + c) * HW + pix] : 0.0f;
            const float It = fmaf(T, a.background, I[c]);
            float yv;
            if constexpr (EPI == kEpiSart) yv = (F - It) * inv;
            else if constexpr (EPI == kEpiMlem) yv = It > 0.0f ? F / It : 1.0f;
            else yv = F - It;
            yo[c] = m != 0.0f ? yv : 0.0f;
            if (in_image) r2 = fmaf(F - It, F - It, r2);
        }
        // residuals per ray, one 16-byte store for three channels
        if (in_image) {
            if constexpr (C == 3) reinterpret_cast<float4 *>(a.out)[r] = make_float4(yo[0], yo[1], yo[2], 0.0f);
            else a.out[r] = yo[0];
        }
        if (a.err) {
            // fixed-order butterfly over the tile's 64 rays; lane 0 stores it
            float e0 = m != 0.0f ? r2 : 0.0f, e1 = m != 0.0f ? (float)C : 0.0f;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                e0 += __shfl_xor(e0, off, 64);
                e1 += __shfl_xor(e1, off, 64);
            }
            if (lane == 0) a.err[slot] = make_float2(e0, e1);
        }
    }
}

template <int C, bool EMIS, bool SCAT, bool WRITE_G, int EPI>
__global__ __launch_bounds__(kBlock) void render_kernel(
    RenderArgs a)
{
    render_body<C, EMIS, SCAT, WRITE_G, EPI>(a, blockIdx.x);
}

// Job of a block in a batched launch: prefix[j] is the first block of job j.
__device__ __forceinline__ int batch_job(const int *prefix, int n, int b)
{
    int j = 0;
    while (j + 1 < n && prefix[j + 1] <= b) ++j;
    return j;
}

// One launch covering the tiles of several independent jobs (plans).
template <int C, bool EMIS, bool SCAT, bool WRITE_G, int EPI>
__global__ __launch_bounds__(kBlock) void render_batch_kernel(
    const RenderArgs *args, const int *prefix, int n)
{
    const int j = batch_job(prefix, n, blockIdx.x);
    render_body<C, EMIS, SCAT, WRITE_G, EPI>(args[j], blockIdx.x - prefix[j]);
}

// --------------------------------------------------------- K6 adjoint march

// dphi/dx = (e^-x (1 + x) - 1) / x^2 given e = e^-x; Taylor series below 0.25.
__device__ __forceinline__ float dphi_f(float x, float e)
{
    const float ser =
        fmaf(x, fmaf(x, fmaf(x, fmaf(x, fmaf(x, 1.0f / 840.0f, -1.0f / 144.0f), 1.0f / 30.0f), -0.125f),
                  1.0f / 3.0f),
             -0.5f);
    const float dir = (fmaf(e, x, e) - 1.0f) * __builtin_amdgcn_rcpf(x * x);
    return x < 0.25f ? ser : dir;
}

struct GradArgs {
    const float4 *rayA, *rayB;
    const uint32_t *tile_off;  // first slot of each tile in the per-sample buffers
    const int32_t *tile_order;
    int n_launch;
    const float *vol;
    const float4 *scat;
    int scat_vstride;     // as in RenderArgs
    const double *exit_tau;  // [V][H][W] optical depth at the exit
    const float *dI;      // dL/dI [V][C][H][W]
    float2 *gq;           // per-sample outputs (g_k, q_k), [tile][K - 1 - k][lane]: row j = step j
    int W, H, tiles_x, tiles_per_view;
    int nx, ny, nz, M;
    float ds, albedo, background;
    float s_scale[3];
};

// Reverse march of one pixel ray for the gradient of a loss with dL/dI given.
// Starting from the stored exit optical depth tau_K = sum_k a_k (FP64), each
// step takes a_k off it and recovers T_k = exp(-tau_k): a ray whose exit
// transmittance underflows FP32 (tau_K beyond about 87) still gets the
// exact T_k wherever T_k itself is representable. It re-samples the volume
// and writes
//   g_k = T_k Delta_k phi(a_k)                              (dI/d eps_k)
//   q_k = sum_c dL/dI_c [T_k (albedo S_c Delta_k phi + j_c Delta_k^2 phi')
//                        - Delta_k R_c]                      (dL/d sigma_k)
// with R_c the radiance of everything behind sample k; nothing per sample is
// kept from the forward pass. sigma_k = max(0, trilinear) passes the
// derivative where the trilinear value is >= 0. Step j stores every ray's
// sample in row j of the tile (sample K - 1 - j of a ray with K samples), so
// the wave writes one contiguous row per step.
template <int C, bool SCAT>
__global__ __launch_bounds__(kBlock) void adjoint_march_kernel(GradArgs a)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int slot = blockIdx.x * 4 + wave;
    if (slot >= a.n_launch) return;
    // every lane of the wave reads the same entry: keep the tile (and so the
    // view and the per-view in-scatter grid address) in scalar registers
    const int tile = __builtin_amdgcn_readfirstlane(a.tile_order[slot]);
    if (tile < 0) return;  // an empty slot of an XCD's band
    const int v = tile / a.tiles_per_view, t = tile - v * a.tiles_per_view;
    const int ty = t / a.tiles_x, tx = t - ty * a.tiles_x;
    const int px = tx * kTile + (lane & 7), py = ty * kTile + (lane >> 3);
    // lanes past the image edge or missing the box stay for the window loads
    const bool in_image = px < a.W && py < a.H;
    const int HW = a.W * a.H;
    const int pix = in_image ? py * a.W + px : 0;
    const int r = v * HW + pix;
    const float4 A = a.rayA[r], B = a.rayB[r];
    const int K = in_image ? __float_as_int(B.w) : 0;
    const int nx = a.nx, nxy = a.nx * a.ny;
    constexpr int elem = C == 3 ? 16 : 8;
    const __amdgpu_buffer_rsrc_t vr = make_rsrc(a.vol, (int64_t)nxy * a.nz * elem);
    int coff[8];
    corner_offsets(nx, nxy, elem, coff);
    const int M = a.M, MM = a.M * a.M;
    const __amdgpu_buffer_rsrc_t sr =
        make_rsrc(a.scat + (int64_t)v * a.scat_vstride, SCAT ? (int64_t)MM * M * 16 : 16);
    int soff[8];
    corner_offsets(M, MM, 16, soff);
    float y[C], R[C];
    double tau = a.exit_tau[r];
    const float TK = __expf(-(float)tau);
#pragma unroll
    for (int c = 0; c < C; ++c) {
        y[c] = a.dI[(v * C + c) * HW + pix];
        R[c] = TK * a.background;
    }
    float2 *gqp = a.gq + a.tile_off[tile] + lane;
    ScatCorners scc;
    __shared__ typename Packed<C>::T win_lds[4][kWinSlots];
    VolWindow<C> win;
    win.lds = win_lds[wave];
    {
        // the march runs back to front: the window trails along -direction
        float sx = B.x, sy = B.y, sz = B.z;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            sx += __shfl_xor(sx, off, 64);
            sy += __shfl_xor(sy, off, 64);
            sz += __shfl_xor(sz, off, 64);
        }
        win.fx = sx < 0.0f;
        win.fy = sy < 0.0f;
        win.fz = sz < 0.0f;
    }
    // all lanes step together; step j takes sample K - 1 - j of each ray
    const int Kw = wave_max(K);
    for (int j = 0; j < Kw; ++j) {
        const int k = K - 1 - j;
        const bool act = k >= 0;
        float s = 0.0f, len = 0.0f;
        if (act) segment_of(k, K, A.w, a.ds, s, len);
        const float x = fmaf(s, B.x, A.x), yy = fmaf(s, B.y, A.y), z = fmaf(s, B.z, A.z);
        int ix, iy, iz;
        float fx, fy, fz;
        cell_of(x, a.nx, ix, fx);
        cell_of(yy, a.ny, iy, fy);
        cell_of(z, a.nz, iz, fz);
        const bool in_win = win.update(act, ix, iy, iz, vr, a.nx, a.ny, a.nz, lane);
        if (!act) continue;
        float w[8];
        tri_weights(fx, fy, fz, w);
        float em[C], sraw;
        if (in_win) {
            win.sample(ix, iy, iz, w, em, sraw);
        } else {
            VolCorners<C> vcc;
            const int base = (int)(__umul24(iz, nxy) + __umul24(iy, nx)) + ix;
            sample_volume_rsrc<C>(vr, coff, base * elem, w, vcc, em, sraw);
        }
        const float sig = fmaxf(sraw, 0.0f);
        float S[3] = {0.f, 0.f, 0.f};
        if constexpr (SCAT) {
            int jx, jy, jz;
            float gx, gy, gz;
            cell_of(x * a.s_scale[0], M, jx, gx);
            cell_of(yy * a.s_scale[1], M, jy, gy);
            cell_of(z * a.s_scale[2], M, jz, gz);
            float ws[8];
            tri_weights(gx, gy, gz, ws);
            const int sb = ((int)(__umul24(jz, MM) + __umul24(jy, M)) + jx) * 16;
            scat_sample(sr, soff, sb, ws, scc, S);
            const float as = a.albedo * sig;
#pragma unroll
            for (int c = 0; c < C; ++c) em[c] = fmaf(as, S[c], em[c]);
        }
        const float xo = sig * len;
        float e;
        const float ph = phi_exp(xo, e);
        const float dph = dphi_f(xo, e);
        tau -= (double)xo;
        const float T = __expf(-(float)tau);  // transmittance in front of sample k
        const float gk = T * len * ph;
        float qk = 0.0f;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const float dc = T * len * fmaf(a.albedo * S[c], ph, em[c] * len * dph);
            qk = fmaf(y[c], fmaf(-len, R[c], dc), qk);
            R[c] = fmaf(gk, em[c], R[c]);
        }
        gqp[j * kTileRays] = make_float2(gk, sraw >= 0.0f ? qk : 0.0f);
    }
}

// ----------------------------------------------------------- K2 in-scatter

// In-scatter passes. A packed volume of at most kScatSlabBytes is marched in
// one pass by all XCDs. A larger one is cut into 8 slabs along z and XCD x
// marches slab x only, so its L2 (4 MB) holds one slab instead of the
// volume: on the 128^3 colour workload (33 MB) the march takes 0.56 ms
// instead of 0.82 ms with 4 slabs of 8 MB marched by all XCDs together; with
// the same sample count, a 64^3 volume (4 MB) takes 0.29 ms in one pass and
// 0.37 ms in 8 slab passes.
constexpr int64_t kScatSlabBytes = 8ll << 20;
// With 8 slabs, pass 4 is the last: every ray still alive then marches to
// its end in that pass (from slab 4 up or slab 3 down), leaving passes 5-7
// to no one. Those passes would hold few rays each, too few to fill the
// chip; ending at pass 4 takes the 128^3 colour march from 0.56 ms to
// 0.53 ms (ending at pass 2, 3, 5 or 6: 0.55, 0.57, 0.54, 0.55 ms).
constexpr int kScatFinalPass = 4;

struct ScatArgs {
    const float *vol;
    const float4 *dirs;  // unit directions in voxel units per world unit (xyz)
    float *dpart;        // per-direction sums [ndirs][C][M^3]
    int *kstate;         // per (direction, node): next sample to march [ndirs][M^3]
    float *tstate;       // per (direction, node): transmittance so far [ndirs][M^3]
    int pass, npass;     // slab pass and number of passes
    float slab_h;        // slab thickness along z (fine grid units)
    float4 *scat;        // packed output (rgb, 0)
    float *planar;       // optional [C][M^3]
    int nx, ny, nz, M, ndirs;
    int nbricks, blocks_per_dir, dirs_per_xcd;
    int xslab;           // 1: XCD x owns slab x (8 slabs); 0: all XCDs march one slab per pass
    int nup;             // directions 0 .. nup-1 point up (u.z >= 0), the rest down
    int bz_lo[8], bz_hi[8];  // xslab: node-brick layers that hold the nodes starting in each slab
    float p_scale[3];    // in-scatter node index -> fine grid coords
    float ds;            // world step
    float inv_ndirs;
    // anisotropic phase function (one grid per view)
    const rte_camera *cams;
    const double *dirs_world;  // [ndirs][3] unit directions, world frame
    int V;
    double phase_g;
    double lo[3], hs[3];       // world position of in-scatter node m: lo + m * hs
};

// March in slab passes (a wave = one 4x4x4 brick of nodes and one
// direction, a block = four such waves). Every ray stops at the first sample
// beyond its slab and keeps the next sample index, the transmittance and the
// partial sums for the next pass; every sample is taken exactly once, in the
// same order and arithmetic as a single march, so the sums are those of one
// march. Two schedules:
//  * xslab: 8 slabs, XCD x (blocks b with b % 8 == x) owns slab x. Rays are
//    monotone in z and cross one slab per pass, so in pass p XCD x takes the
//    up-going rays of the nodes that start in slab x - p and the down-going
//    rays of those starting in slab x + p; each XCD's working set is its slab.
//  * otherwise (one pass): XCD x takes directions x, x + 8, ... and every
//    ray marches to the box exit (the one slab is the edge slab).
// The march is software-pipelined: the corner loads of the next sample are
// issued before the current sample is accumulated (the loads wait on memory,
// the sums on nothing but the loads). Each (direction, node) sum is stored;
// the directions are added in order by inscatter_reduce_kernel.
template <int C>
__device__ __forceinline__ void inscatter_march_body(const ScatArgs &a, const int pass, const int blk)
{
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int x = blk & 7, j = blk >> 3;
    const int M = a.M, bm = (M + 3) >> 2;
    int d, bx, by, bz, start = 0;
    if (a.xslab) {
        // XCD x marches slab x: in pass p, the up-going rays of the nodes that
        // start in slab x - p and the down-going rays of those starting in
        // slab x + p (a ray crosses one slab per pass)
        const int s_up = x - pass, s_dn = x + pass;
        const int bxy = bm * bm;
        const int nl_up = s_up >= 0 ? max(a.bz_hi[s_up] - a.bz_lo[s_up] + 1, 0) : 0;
        const int nl_dn = s_dn < a.npass ? max(a.bz_hi[s_dn] - a.bz_lo[s_dn] + 1, 0) : 0;
        const int items_up = a.nup * nl_up * bxy, items_dn = (a.ndirs - a.nup) * nl_dn * bxy;
        int item = j * 4 + w, rem;
        if (item < items_up) {
            d = item / (nl_up * bxy);
            rem = item - d * (nl_up * bxy);
            bz = a.bz_lo[s_up] + rem / bxy;
            start = s_up;
        } else {
            item -= items_up;
            if (item >= items_dn) return;
            const int dd = item / (nl_dn * bxy);
            rem = item - dd * (nl_dn * bxy);
            d = a.nup + dd;
            bz = a.bz_lo[s_dn] + rem / bxy;
            start = s_dn;
        }
        const int bxyi = rem % bxy;
        bx = bxyi % bm;
        by = bxyi / bm;
    } else {
        d = x + 8 * (j / a.blocks_per_dir);
        const int brick = (j % a.blocks_per_dir) * 4 + w;
        if (d >= a.ndirs || brick >= a.nbricks) return;
        bx = brick % bm;
        by = (brick / bm) % bm;
        bz = brick / (bm * bm);
    }
    const int mx = bx * 4 + (l & 3), my = by * 4 + ((l >> 2) & 3), mz = bz * 4 + (l >> 4);
    if (mx >= M || my >= M || mz >= M) return;
    const float px = (float)mx * a.p_scale[0], py = (float)my * a.p_scale[1],
                pz = (float)mz * a.p_scale[2];
    if (a.xslab && min(a.npass - 1, (int)(pz / a.slab_h)) != start) return;  // the node starts in another slab
    const float tx = (float)(a.nx - 1), ty = (float)(a.ny - 1), tz = (float)(a.nz - 1);
    const int nx = a.nx, nxy = a.nx * a.ny;
    constexpr int elem = C == 3 ? 16 : 8;
    const __amdgpu_buffer_rsrc_t vr = make_rsrc(a.vol, (int64_t)nxy * a.nz * elem);
    int coff[8];
    corner_offsets(nx, nxy, elem, coff);
    const float4 u = a.dirs[d];
    // exit distance from an interior point (world units)
    float ell = INFINITY;
    if (u.x > 0.f) ell = fminf(ell, (tx - px) / u.x);
    if (u.x < 0.f) ell = fminf(ell, -px / u.x);
    if (u.y > 0.f) ell = fminf(ell, (ty - py) / u.y);
    if (u.y < 0.f) ell = fminf(ell, -py / u.y);
    if (u.z > 0.f) ell = fminf(ell, (tz - pz) / u.z);
    if (u.z < 0.f) ell = fminf(ell, -pz / u.z);
    ell = fmaxf(ell, 0.0f);
    const int K = ell > 0.0f ? (int)ceilf(ell / a.ds) : 0;
    const int m3 = M * M * M;
    const int m = (mz * M + my) * M + mx;
    const int64_t st = (int64_t)d * m3 + m;
    float acc[C];
    float T = 1.0f;
    int k0 = 0;
    if (pass == 0) {
#pragma unroll
        for (int c = 0; c < C; ++c) acc[c] = 0.0f;
    } else {
        k0 = a.kstate[st];
        if (k0 >= K) return;  // this ray has left the box
        T = a.tstate[st];
#pragma unroll
        for (int c = 0; c < C; ++c) acc[c] = a.dpart[(int64_t)(d * C + c) * m3 + m];
    }
    const bool up = u.z >= 0.0f;
    // the slab marched in this pass; the edge slab, and any slab in the final
    // pass, takes every remaining sample
    const int slab = a.xslab ? x : (up ? pass : a.npass - 1 - pass);
    const bool last = a.xslab ? ((up ? slab == a.npass - 1 : slab == 0) || pass == kScatFinalPass)
                              : pass == a.npass - 1;
    const float zlo = (float)slab * a.slab_h, zhi = (float)(slab + 1) * a.slab_h;
    // software pipeline: the corner loads of sample k + 1 are in flight
    // while sample k is accumulated (the positions do not depend on the sums)
    using PT = typename Packed<C>::T;
    auto locate = [&](int kk, float &len, float &zs, int &base, float &fx, float &fy, float &fz) {
        float s;
        segment_of(kk, K, ell, a.ds, s, len);
        zs = fmaf(s, u.z, pz);
        int ix, iy, iz;
        cell_of(fmaf(s, u.x, px), a.nx, ix, fx);
        cell_of(fmaf(s, u.y, py), a.ny, iy, fy);
        cell_of(zs, a.nz, iz, fz);
        base = ((int)(__umul24(iz, nxy) + __umul24(iy, nx)) + ix) * elem;
    };
    auto fetch = [&](int base, PT v[8]) {
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            if constexpr (C == 3) v[c] = bload4(vr, base, coff[c]);
            else v[c] = bload2(vr, base, coff[c]);
        }
    };
    int k = k0;
    PT cur[8];
    float len = 0.f, zs = 0.f, fx = 0.f, fy = 0.f, fz = 0.f;
    if (k < K) {
        int base;
        locate(k, len, zs, base, fx, fy, fz);
        fetch(base, cur);
    }
    for (; k < K; ++k) {
        if (!last && (up ? zs >= zhi : zs < zlo)) break;
        PT nxt[8];
        float len2 = 0.f, zs2 = 0.f, fx2 = 0.f, fy2 = 0.f, fz2 = 0.f;
        int base2 = 0;
        if (k + 1 < K) {
            locate(k + 1, len2, zs2, base2, fx2, fy2, fz2);
            // a sample beyond this slab is taken by the next pass: the loop
            // stops before using it, so it is not fetched here
            if (last || !(up ? zs2 >= zhi : zs2 < zlo)) fetch(base2, nxt);
        }
        float wt[8];
        tri_weights(fx, fy, fz, wt);
        float em[C], sig;
        interp_corners<C>(cur, wt, em, sig);
        sig = fmaxf(sig, 0.0f);
        float e;
        const float wg = T * len * phi_exp(sig * len, e);
#pragma unroll
        for (int c = 0; c < C; ++c) acc[c] = fmaf(wg, em[c], acc[c]);
        T *= e;
#pragma unroll
        for (int c = 0; c < 8; ++c) cur[c] = nxt[c];
        len = len2;
        zs = zs2;
        fx = fx2;
        fy = fy2;
        fz = fz2;
    }
    if (k == k0 && pass > 0) return;  // nothing in this slab: the state stands
    if (!last) {
        a.kstate[st] = k;
        a.tstate[st] = T;
    }
#pragma unroll
    for (int c = 0; c < C; ++c) a.dpart[(int64_t)(d * C + c) * m3 + m] = acc[c];
}

template <int C>
__global__ __launch_bounds__(kBlock) void inscatter_march_kernel(ScatArgs a)
{
    inscatter_march_body<C>(a, a.pass, blockIdx.x);
}

// One pass of several plans' in-scatter marches in one launch: prefix[j] is
// the first block of plan j (a multiple of 8, so every block keeps the XCD it
// has in the plan's own launch); plans without this pass have no blocks.
template <int C>
__global__ __launch_bounds__(kBlock) void inscatter_march_batch_kernel(const ScatArgs *args, const int *prefix,
                                                                      int n, int pass)
{
    const int j = batch_job(prefix, n, blockIdx.x);
    inscatter_march_body<C>(args[j], pass, blockIdx.x - prefix[j]);
}

// S_c(node) = (1 / ndirs) sum_d, the directions added in index order. Small
// blocks: a 32^3 grid is 512 of them, enough to reach every CU.
constexpr int kReduceBlock = 64;
template <int C>
__device__ __forceinline__ void inscatter_reduce_body(const ScatArgs &a, const int blk)
{
    const int m3 = a.M * a.M * a.M;
    const int m = blk * kReduceBlock + threadIdx.x;
    if (m >= m3) return;
    float tot[C];
#pragma unroll
    for (int c = 0; c < C; ++c) tot[c] = 0.0f;
#pragma unroll 4
    for (int d = 0; d < a.ndirs; ++d)
#pragma unroll
        for (int c = 0; c < C; ++c) tot[c] += a.dpart[(int64_t)(d * C + c) * m3 + m];
#pragma unroll
    for (int c = 0; c < C; ++c) tot[c] *= a.inv_ndirs;
    float4 o = make_float4(tot[0], 0.f, 0.f, 0.f);
    if constexpr (C == 3) {
        o.y = tot[1];
        o.z = tot[2];
    }
    a.scat[m] = o;
    if (a.planar) {
        a.planar[m] = o.x;
        if constexpr (C == 3) {
            a.planar[m3 + m] = o.y;
            a.planar[2 * m3 + m] = o.z;
        }
    }
}

template <int C>
__global__ __launch_bounds__(kReduceBlock) void inscatter_reduce_kernel(ScatArgs a)
{
    inscatter_reduce_body<C>(a, blockIdx.x);
}

template <int C>
__global__ __launch_bounds__(kReduceBlock) void inscatter_reduce_batch_kernel(const ScatArgs *args, const int *prefix,
                                                                             int n)
{
    const int j = batch_job(prefix, n, blockIdx.x);
    inscatter_reduce_body<C>(args[j], blockIdx.x - prefix[j]);
}

// Henyey-Greenstein in-scattering (Eq. 9, g != 0): view v sees at node p the
// incident radiance of every direction u_d weighted by p(w, u_d), w the
// direction from p to the camera centre (the direction the scattered light
// travels; u_d points to where the light comes from), the weights normalised
// over the directions (a radiance equal in every direction scatters into
// itself). The weights are evaluated in FP64: near |g| -> 1 the denominator
// 1 + g^2 + 2 g cos is a difference of nearly equal terms. One work-item per
// (node, view); directions are added in index order.
template <int C>
__device__ __forceinline__ void inscatter_phase_reduce_body(const ScatArgs &a, const int blk, const int v)
{
    const int m3 = a.M * a.M * a.M;
    const int m = blk * kBlock + threadIdx.x;
    if (m >= m3 || v >= a.V) return;
    const int M = a.M, mx = m % M, my = (m / M) % M, mz = m / (M * M);
    const rte_camera &cam = a.cams[v];
    double w[3], nrm2 = 0.0;
    const int ms[3] = {mx, my, mz};
    for (int i = 0; i < 3; ++i) {
        const double o = -(cam.R[i] * cam.t[0] + cam.R[3 + i] * cam.t[1] + cam.R[6 + i] * cam.t[2]);
        w[i] = o - (a.lo[i] + (double)ms[i] * a.hs[i]);
        nrm2 += w[i] * w[i];
    }
    const double inv = nrm2 > 0.0 ? 1.0 / sqrt(nrm2) : 0.0;
    const double g = a.phase_g, g2 = g * g;
    double num[C], den = 0.0;
#pragma unroll
    for (int c = 0; c < C; ++c) num[c] = 0.0;
    for (int d = 0; d < a.ndirs; ++d) {
        double W = 1.0;
        if (nrm2 > 0.0) {
            const double *u = a.dirs_world + 3 * d;
            const double cs = (w[0] * u[0] + w[1] * u[1] + w[2] * u[2]) * inv;
            const double x = 1.0 + g2 + 2.0 * g * cs;
            W = (1.0 - g2) / (x * sqrt(x));
        }
        den += W;
#pragma unroll
        for (int c = 0; c < C; ++c) num[c] += W * (double)a.dpart[(int64_t)(d * C + c) * m3 + m];
    }
    float out[C];
#pragma unroll
    for (int c = 0; c < C; ++c) out[c] = (float)(num[c] / den);
    float4 o = make_float4(out[0], 0.f, 0.f, 0.f);
    if constexpr (C == 3) {
        o.y = out[1];
        o.z = out[2];
    }
    a.scat[(int64_t)v * m3 + m] = o;
    if (a.planar) {
#pragma unroll
        for (int c = 0; c < C; ++c) a.planar[(int64_t)(v * C + c) * m3 + m] = out[c];
    }
}

template <int C>
__global__ __launch_bounds__(kBlock) void inscatter_phase_reduce_kernel(ScatArgs a)
{
    inscatter_phase_reduce_body<C>(a, blockIdx.x, blockIdx.y);
}

// Several plans' per-view reductions in one launch: plan j has
// ceil(M^3 / kBlock) blocks per view, views one after another.
template <int C>
__global__ __launch_bounds__(kBlock) void inscatter_phase_reduce_batch_kernel(const ScatArgs *args,
                                                                             const int *prefix, int n)
{
    const int j = batch_job(prefix, n, blockIdx.x);
    const ScatArgs &a = args[j];
    const int per_view = (a.M * a.M * a.M + kBlock - 1) / kBlock;
    const int local = blockIdx.x - prefix[j];
    inscatter_phase_reduce_body<C>(a, local % per_view, local / per_view);
}

// ---------------------------------------------------------------- K3 gather

struct GatherArgs {
    const float4 *rayA, *rayB;
    const uint32_t *tile_off;  // first slot of each tile in the per-sample buffers
    const float *g;
    const float *q;        // gradient mode: per-sample (g_k, q_k) pairs, float2 [tile][K - 1 - k][lane]
    const float *y;        // residual per ray [V][H][W]: float4 (RGB, pad) for 3 channels, float for 1
    const ViewProj *proj;
    float *part;           // [8][acc][cells]
    int V, W, H, tiles_x, tiles_per_view;
    int nx, ny, nz;
    int bx, by, bz, nb8;   // bricks of 8x8x4 cells
    int ncells;
    float ds, inv_ds;
    float alpha_l, alpha_d, log2_keep;  // paper mode
    float g_sigma;                      // paper mode: spread of the gains G(s)
    uint32_t seed_lo, seed_hi;
    int iteration;
    const float *rowmask;               // optional [V][H][W]: rays with 0 are skipped (cols, hull, adjoint+cols)
    int view0, view_step;               // views view0, view0 + view_step, ... (ordered subsets)
};

constexpr float kBoxPad = 1e-3f;   // voxels: cell box padding for FP32 sample positions
constexpr float kPixPad = 2e-3f;   // pixels: projection rounding allowance

template <int C, int MODE>
struct GatherAcc {
    static constexpr int N = MODE == kGatherHull ? 2
                             : ((MODE == kGatherAdjointCols || MODE == kGatherGrad) ? C + 1 : C);
};

// Each work-item owns one cell (voxel) c and gathers every sample that the
// render march placed in c: for each view it projects the (slightly padded)
// cell box to a pixel rectangle, intersects each candidate pixel ray with the
// box to bound the sample indices, and re-derives every candidate sample's
// position exactly as the render did; only samples whose cell is c are kept.
// The trilinear weights of the sample distribute its contribution to the
// cell's 8 corners. Sums run in a fixed order: views, then pixels row-major,
// then samples.
template <int C, int MODE>
__device__ __forceinline__ void gather_body(const GatherArgs &a, int b)
{
    constexpr int NA = GatherAcc<C, MODE>::N;
    if (b >= a.bx * a.by * a.bz) return;
    const int bxi = b % a.bx, byi = (b / a.bx) % a.by, bzi = b / (a.bx * a.by);
    const int cx = bxi * 8 + (threadIdx.x & 7);
    const int cy = byi * 8 + ((threadIdx.x >> 3) & 7);
    const int cz = bzi * 4 + (threadIdx.x >> 6);
    // work-items past the grid's last cell gather nothing but stay for the
    // brick's key-point sums
    const bool valid = cx < a.nx - 1 && cy < a.ny - 1 && cz < a.nz - 1;

    float acc[8][NA];
#pragma unroll
    for (int c = 0; c < 8; ++c)
#pragma unroll
        for (int q = 0; q < NA; ++q) acc[c][q] = 0.0f;

    const float lo[3] = {(float)cx - kBoxPad, (float)cy - kBoxPad, (float)cz - kBoxPad};
    const float hi[3] = {(float)cx + 1.0f + kBoxPad, (float)cy + 1.0f + kBoxPad,
                         (float)cz + 1.0f + kBoxPad};
    const int HW = a.W * a.H;
    uint64_t hull_bits = 0;

    for (int v = a.view0; valid && v < a.V; v += a.view_step) {
        const float *P = a.proj[v].P;
        bool found = false;  // hull mode: this view already tags the cell
        // project the 8 corners of the padded box
        float umin = INFINITY, umax = -INFINITY, vmin = INFINITY, vmax = -INFINITY;
        bool behind = false;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const float X = (c & 1) ? hi[0] : lo[0];
            const float Y = (c & 2) ? hi[1] : lo[1];
            const float Z = (c & 4) ? hi[2] : lo[2];
            const float hu = fmaf(P[0], X, fmaf(P[1], Y, fmaf(P[2], Z, P[3])));
            const float hv = fmaf(P[4], X, fmaf(P[5], Y, fmaf(P[6], Z, P[7])));
            const float hw = fmaf(P[8], X, fmaf(P[9], Y, fmaf(P[10], Z, P[11])));
            behind = behind || !(hw > 1e-6f);
            const float iw = __builtin_amdgcn_rcpf(hw);
            const float u = hu * iw, vv = hv * iw;
            umin = fminf(umin, u);
            umax = fmaxf(umax, u);
            vmin = fminf(vmin, vv);
            vmax = fmaxf(vmax, vv);
        }
        int u0 = 0, u1 = a.W - 1, v0 = 0, v1 = a.H - 1;
        if (!behind) {
            u0 = max(u0, (int)ceilf(umin - 0.5f - kPixPad));
            u1 = min(u1, (int)floorf(umax - 0.5f + kPixPad));
            v0 = max(v0, (int)ceilf(vmin - 0.5f - kPixPad));
            v1 = min(v1, (int)floorf(vmax - 0.5f + kPixPad));
        }
        // one candidate pixel ray: slab test against the padded cell, then
        // every sample of the ray that the render placed in this cell
        constexpr bool kReadsG = MODE == kGatherAdjoint || MODE == kGatherAdjointCols || MODE == kGatherGrad;
        auto tile_of = [&](int px, int py) { return v * a.tiles_per_view + (py >> 3) * a.tiles_x + (px >> 3); };
        // toff: first slot of the candidate's tile in the per-sample buffers
        // (loaded with the candidate's ray, one candidate ahead)
        auto candidate = [&](int px, int py, int r, const float4 &A, const float4 &B, uint32_t toff) {
            if ((MODE == kGatherHull || MODE == kGatherAdjointCols) && a.rowmask &&
                a.rowmask[r] == 0.0f)
                return;
            const int K = __float_as_int(B.w);
            if (K == 0) return;
            // slab test against the padded cell box, in ray offset s
            float s_in = 0.0f, s_out = A.w;
            {
                const float pa[3] = {A.x, A.y, A.z};
                const float da[3] = {B.x, B.y, B.z};
#pragma unroll
                for (int ax = 0; ax < 3; ++ax) {
                    const float id = __builtin_amdgcn_rcpf(da[ax]);
                    const float t0 = (lo[ax] - pa[ax]) * id, t1 = (hi[ax] - pa[ax]) * id;
                    s_in = fmaxf(s_in, fminf(t0, t1));
                    s_out = fminf(s_out, fmaxf(t0, t1));
                }
            }
            if (!(s_out >= s_in)) return;
            // samples k < K-1 sit at s = (k + 1/2) ds; the last one lies in
            // [(K-1) ds, L]. The padded box keeps every sample the render
            // placed in this cell inside [s_in, s_out] despite rounding.
            const int k_lo = max(0, (int)ceilf(fmaf(s_in, a.inv_ds, -0.5f)));
            int k_hi = min(K - 2, (int)floorf(fmaf(s_out, a.inv_ds, -0.5f)));
            if (s_out >= (float)(K - 1) * a.ds) k_hi = K - 1;
            if (k_lo > k_hi) return;
            float yv[C];
            if constexpr (MODE != kGatherHull) {
                if constexpr (C == 3) {
                    const float4 y4 = reinterpret_cast<const float4 *>(a.y)[r];
                    yv[0] = y4.x;
                    yv[1] = y4.y;
                    yv[2] = y4.z;
                } else {
                    yv[0] = a.y[r];
                }
            }
            // weights of the candidate's samples: the group holding k_lo is
            // loaded here, the next one only if the samples run into it
            const uint32_t pl = (uint32_t)((py & 7) * 8 + (px & 7));
            constexpr bool kGroups = MODE == kGatherAdjoint || MODE == kGatherAdjointCols;
            const float4 *g4 = reinterpret_cast<const float4 *>(a.g);
            const uint32_t gbase = toff / kGroup + pl;  // group 0 of this pixel, < 2^30
            int gi = k_lo / kGroup;
            float4 G = make_float4(0.f, 0.f, 0.f, 0.f);
            if constexpr (kGroups) G = g4[gbase + (uint32_t)gi * kTileRays];
            for (int k = k_lo; k <= k_hi; ++k) {
                float s, len;
                segment_of(k, K, A.w, a.ds, s, len);
                int ix, iy, iz;
                float fx, fy, fz;
                cell_of(fmaf(s, B.x, A.x), a.nx, ix, fx);
                cell_of(fmaf(s, B.y, A.y), a.ny, iy, fy);
                cell_of(fmaf(s, B.z, A.z), a.nz, iz, fz);
                if (ix != cx || iy != cy || iz != cz) continue;
                if constexpr (MODE == kGatherHull) {
                    hull_bits |= (uint64_t)1 << v;
                    found = true;
                    break;
                } else if constexpr (MODE == kGatherPaper) {
                    float keep = exp2f((float)k * a.log2_keep);
                    if (a.g_sigma != 0.0f)
                        keep *= sample_gain(a.seed_lo, a.seed_hi, a.iteration, v, py * a.W + px, k, a.g_sigma);
#pragma unroll
                    for (int c = 0; c < 8; ++c) {
                        const float ddx = fx - (float)(c & 1);
                        const float ddy = fy - (float)((c >> 1) & 1);
                        const float ddz = fz - (float)((c >> 2) & 1);
                        const float D = sqrtf(fmaf(ddx, ddx, fmaf(ddy, ddy, ddz * ddz)));
                        const float amp = a.alpha_l * keep * __expf(-a.alpha_d * D);
#pragma unroll
                        for (int q = 0; q < C; ++q) acc[c][q] = fmaf(amp, yv[q], acc[c][q]);
                    }
                } else {
                    float gk, qk = 0.0f;
                    if constexpr (MODE == kGatherGrad) {
                        // the adjoint march stores sample k in row K - 1 - k
                        const float2 gq = reinterpret_cast<const float2 *>(a.q)[toff + pl + (K - 1 - k) * kTileRays];
                        gk = gq.x;
                        qk = gq.y;
                    } else {
                        if (k / kGroup != gi) {
                            gi = k / kGroup;
                            G = g4[gbase + (uint32_t)gi * kTileRays];
                        }
                        // two selects, no branches
                        const float g01 = (k & 1) ? G.y : G.x;
                        const float g23 = (k & 1) ? G.w : G.z;
                        gk = (k & 2) ? g23 : g01;
                    }
                    float w[8];
                    tri_weights(fx, fy, fz, w);
                    if constexpr (MODE == kGatherGrad) {
                        float gy[C];
#pragma unroll
                        for (int qq = 0; qq < C; ++qq) gy[qq] = gk * yv[qq];
#pragma unroll
                        for (int c = 0; c < 8; ++c) {
#pragma unroll
                            for (int qq = 0; qq < C; ++qq) acc[c][qq] = fmaf(gy[qq], w[c], acc[c][qq]);
                            acc[c][C] = fmaf(qk, w[c], acc[c][C]);
                        }
                    } else {
                        float gy[C];
#pragma unroll
                        for (int q = 0; q < C; ++q) gy[q] = gk * yv[q];
#pragma unroll
                        for (int c = 0; c < 8; ++c) {
#pragma unroll
                            for (int q = 0; q < C; ++q) acc[c][q] = fmaf(gy[q], w[c], acc[c][q]);
                            if constexpr (MODE == kGatherAdjointCols)
                                acc[c][C] = fmaf(gk, w[c], acc[c][C]);
                        }
                    }
                }
            }
        };
        // candidate pixels in row-major order; except in the arithmetic-heavy
        // paper mode, the ray of the next candidate is loaded while the
        // current one is processed
        if constexpr (MODE != kGatherPaper) {
            const int ncand = (u1 >= u0 && v1 >= v0) ? (u1 - u0 + 1) * (v1 - v0 + 1) : 0;
            int nxp = u0, nyp = v0;
            float4 An = make_float4(0.f, 0.f, 0.f, 0.f), Bn = An;
            uint32_t Tn = 0;
            if (ncand > 0) {
                const int rn = v * HW + nyp * a.W + nxp;
                An = a.rayA[rn];
                Bn = a.rayB[rn];
                if constexpr (kReadsG) Tn = a.tile_off[tile_of(nxp, nyp)];
            }
            for (int i = 0; i < ncand && !found; ++i) {
                const int px = nxp, py = nyp;
                if (++nxp > u1) {
                    nxp = u0;
                    ++nyp;
                }
                const float4 A = An, B = Bn;
                const uint32_t T = Tn;
                if (i + 1 < ncand) {
                    const int rn = v * HW + nyp * a.W + nxp;
                    An = a.rayA[rn];
                    Bn = a.rayB[rn];
                    if constexpr (kReadsG) Tn = a.tile_off[tile_of(nxp, nyp)];
                }
                candidate(px, py, v * HW + py * a.W + px, A, B, T);
            }
        } else {
            for (int py = v0; py <= v1; ++py) {
                for (int px = u0; px <= u1; ++px) {
                    const int r = v * HW + py * a.W + px;
                    candidate(px, py, r, a.rayA[r], a.rayB[r], 0u);
                }
            }
        }
    }
    if constexpr (MODE == kGatherHull) {
        // brick-major cell index: a wave stores 64 consecutive words per mask
        const int cell = b * kBlock + threadIdx.x;
        if (!valid) return;
        a.part[cell] = __uint_as_float((uint32_t)hull_bits);
        a.part[(int64_t)a.ncells + cell] = __uint_as_float((uint32_t)(hull_bits >> 32));
        return;
    } else {
        // sum the cells' corner contributions into the brick's key points in
        // LDS: in pass e every cell adds its corner e (at offset (e & 1,
        // e >> 1 & 1, e >> 2) from the cell), so no two work-items of a pass
        // meet at one key point, and each key point takes its cells in the
        // fixed order e = 0..7
        __shared__ float nodes[NA * kBrickNodeStride];
        for (int i = threadIdx.x; i < NA * kBrickNodeStride; i += kBlock) nodes[i] = 0.0f;
        __syncthreads();
        // the cell's own corner (0, 0, 0) in the brick's key points
        const int n0 = ((cz - bzi * 4) * kBrickNodesY + (cy - byi * 8)) * kBrickNodesX + (cx - bxi * 8);
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            if (valid) {
                const int n = n0 + ((e >> 2) * kBrickNodesY + ((e >> 1) & 1)) * kBrickNodesX + (e & 1);
#pragma unroll
                for (int q = 0; q < NA; ++q) nodes[q * kBrickNodeStride + n] += acc[e][q];
            }
            __syncthreads();
        }
        float *out = a.part + (int64_t)b * NA * kBrickNodeStride;
        for (int i = threadIdx.x; i < NA * kBrickNodeStride; i += kBlock) out[i] = nodes[i];
    }
}

// Waves per SIMD asked of the compiler: the three-channel adjoint gather
// (the reconstruction's) needs 81 registers with the pipelined candidate
// loop, one above the six-wave budget; at six waves it keeps one value in
// scratch outside the loops and runs 10% faster than at five. The paper-mode
// gather likewise needs 97, one above the five-wave budget.
template <int C, int MODE>
struct GatherOcc {
    static constexpr int W = (C == 3 && MODE == kGatherAdjoint) ? 6 : (C == 3 && MODE == kGatherPaper) ? 5 : 1;
};

template <int C, int MODE>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(GatherOcc<C, MODE>::W))) void gather_kernel(
    GatherArgs a)
{
    gather_body<C, MODE>(a, xcd_remap(blockIdx.x, a.nb8));
}

template <int C, int MODE>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(GatherOcc<C, MODE>::W))) void gather_batch_kernel(
    const GatherArgs *args, const int *prefix, int n)
{
    // blocks dealt round-robin over the XCDs: the jobs' bricks differ in cost
    // (views, image sizes), so contiguous runs per XCD would leave some XCDs
    // with the heaviest job (batched gather 11 -> 23 ms on the serving mix)
    const int j = batch_job(prefix, n, blockIdx.x);
    gather_body<C, MODE>(args[j], blockIdx.x - prefix[j]);
}

// -------------------------------------------------------- assembly + update

struct UpdateArgs {
    const float *part;
    float *vol;          // packed volume (updates)
    float *cols;         // column sums (read by kUpdSart, kUpdMlem)
    float *out;          // delta [C][N] (kUpdDelta, kUpdGrad)
    float *out2;         // extinction gradient [N] (kUpdGrad)
    float *cols_out;     // optional (kUpdSartOS, kUpdMlemOS): also store the column sums here
    const int32_t *inside;  // optional: key points outside the visual hull are not updated
    float *temperature;  // kUpdTemp output
    const float *lut;    // [3][lut_cap]
    int lut_cap, lut_size, fit_channel;
    float t_min, t_max;
    int nx, ny, nz, acc;
    int bx, by, bz;  // gather bricks (8 x 8 x 4 cells) along x, y and z
    int nbx, nby, nblocks;  // update bricks (8 x 8 x 4 key points) along x and y, and their count
    int64_t n;
    float lambda;
    int clamp_nonneg;
};

// Inverse of an increasing LUT row by bisection and linear interpolation.
__device__ __forceinline__ float lut_invert(const float *row, int L, float x, float t_min, float t_max)
{
    if (!(x > row[0])) return t_min;
    if (x >= row[L - 1]) return t_max;
    int lo = 0, hi = L - 1;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (row[mid] <= x) lo = mid; else hi = mid;
    }
    const float f = (x - row[lo]) / (row[hi] - row[lo]);
    const float dT = (t_max - t_min) / (float)(L - 1);
    return fmaf((float)lo + f, dT, t_min);
}

// Sum key point j's partials over the gather bricks that hold it and apply
// the update rule.
template <int C, int MODE>
__device__ __forceinline__ void update_body(const UpdateArgs &a, int blk)
{
    // one block per brick of 8 x 8 x 4 key points: the key points of a
    // gather brick less its upper faces, so a wave's first reads are one
    // contiguous run of the brick's key-point plane
    if (blk >= a.nblocks) return;
    const int jx = (blk % a.nbx) * 8 + (threadIdx.x & 7);
    const int jy = ((blk / a.nbx) % a.nby) * 8 + ((threadIdx.x >> 3) & 7);
    const int jz = (blk / (a.nbx * a.nby)) * 4 + (threadIdx.x >> 6);
    if (jx >= a.nx || jy >= a.ny || jz >= a.nz) return;
    const int64_t j = ((int64_t)jz * a.ny + jy) * a.nx + jx;
    constexpr bool kOS = MODE == kUpdSartOS || MODE == kUpdMlemOS;  // column sums in sum[C]
    constexpr int NQ = MODE == kUpdTemp ? 2 : ((MODE == kUpdGrad || kOS) ? C + 1 : C);
    float sum[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) sum[q] = 0.0f;
    // the brick j falls in first, then (for j on a lower face, edge or
    // corner of it) the bricks below along x, y and z, in a fixed order
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int ox = e & 1, oy = (e >> 1) & 1, oz = e >> 2;
        const int gx = (jx >> 3) - ox, gy = (jy >> 3) - oy, gz = (jz >> 2) - oz;
        const int lx = (jx & 7) + 8 * ox, ly = (jy & 7) + 8 * oy, lz = (jz & 3) + 4 * oz;
        if (lx >= kBrickNodesX || ly >= kBrickNodesY || lz >= kBrickNodesZ) continue;
        if (gx < 0 || gy < 0 || gz < 0 || gx >= a.bx || gy >= a.by || gz >= a.bz) continue;
        const int64_t plane = (int64_t)((gz * a.by + gy) * a.bx + gx) * a.acc;
        const int node = (lz * kBrickNodesY + ly) * kBrickNodesX + lx;
#pragma unroll
        for (int q = 0; q < NQ; ++q) sum[q] += a.part[(plane + q) * kBrickNodeStride + node];
    }
    if constexpr (MODE == kUpdDelta) {
#pragma unroll
        for (int q = 0; q < C; ++q) a.out[q * a.n + j] = sum[q];
    } else if constexpr (MODE == kUpdGrad) {
#pragma unroll
        for (int q = 0; q < C; ++q) a.out[q * a.n + j] = sum[q];
        a.out2[j] = sum[C];
    } else if constexpr (MODE == kUpdTemp) {
        float2 *vol = reinterpret_cast<float2 *>(a.vol);
        float2 p = vol[j];
        float e = p.x;
        const float cs = sum[1];
        if (cs > 0.0f) e = e * fmaf(a.lambda, sum[0] / cs - 1.0f, 1.0f);
        const float *row = a.lut + a.fit_channel * a.lut_cap;
        e = fminf(fmaxf(e, row[0]), row[a.lut_size - 1]);
        a.temperature[j] = lut_invert(row, a.lut_size, e, a.t_min, a.t_max);
    } else {
        if constexpr (kOS) {
            if (a.cols_out) a.cols_out[j] = sum[C];
        }
        if (a.inside && !a.inside[j]) return;
        float cs;
        if constexpr (MODE == kUpdPaper) cs = 1.0f;
        else if constexpr (kOS) cs = sum[C];
        else cs = a.cols[j];
        if (MODE != kUpdPaper && !(cs > 0.0f)) return;
        float em[C];
        if constexpr (C == 3) {
            const float4 p = reinterpret_cast<float4 *>(a.vol)[j];
            em[0] = p.x;
            em[1] = p.y;
            em[2] = p.z;
        } else {
            em[0] = reinterpret_cast<float2 *>(a.vol)[j].x;
        }
#pragma unroll
        for (int q = 0; q < C; ++q) {
            float e = em[q];
            if constexpr (MODE == kUpdSart || MODE == kUpdSartOS) e = fmaf(a.lambda, sum[q] / cs, e);
            if constexpr (MODE == kUpdMlem || MODE == kUpdMlemOS) e = e * fmaf(a.lambda, sum[q] / cs - 1.0f, 1.0f);
            if constexpr (MODE == kUpdPaper) e = e + sum[q];
            if (a.clamp_nonneg) e = fmaxf(e, 0.0f);
            em[q] = e;
        }
        if constexpr (C == 3) {
            float4 *p = reinterpret_cast<float4 *>(a.vol) + j;
            p->x = em[0];
            p->y = em[1];
            p->z = em[2];
        } else {
            reinterpret_cast<float2 *>(a.vol)[j].x = em[0];
        }
    }
}

template <int C, int MODE>
__global__ __launch_bounds__(kBlock) void update_kernel(UpdateArgs a)
{
    // neighbouring bricks on one XCD: the cells on a brick's faces are read
    // by both bricks, so they should meet in the same L2 (colour update
    // 73 -> 59 us, differentiable 0.67 -> 0.55 ms)
    update_body<C, MODE>(a, xcd_remap(blockIdx.x, gridDim.x));
}

template <int C, int MODE>
__global__ __launch_bounds__(kBlock) void update_batch_kernel(const UpdateArgs *args, const int *prefix, int n,
                                                             int total)
{
    // bricks in contiguous runs per XCD, as in update_kernel (every brick
    // costs the same here)
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    if (b >= total) return;
    const int j = batch_job(prefix, n, b);
    update_body<C, MODE>(args[j], b - prefix[j]);
}

// ------------------------------------------------------- K5 temperature map

struct TempArgs {
    const float *T;
    const float *lut;
    float *em;     // planar [3][N] or NULL
    float *sig;    // planar [N] or NULL
    float *vol;    // packed float2 (eps_fit, sigma) or NULL
    int lut_cap, lut_size, fit_channel;
    float t_min, t_max, sigma_max, soot_t0, soot_span;
    int64_t n;
};

__device__ __forceinline__ float lut_lookup(const float *row, int L, float T, float t_min, float t_max)
{
    float pos = (T - t_min) / (t_max - t_min) * (float)(L - 1);
    pos = fminf(fmaxf(pos, 0.0f), (float)(L - 1));
    const int i = min((int)pos, L - 2);
    const float f = pos - (float)i;
    return fmaf(f, row[i + 1] - row[i], row[i]);
}

__global__ __launch_bounds__(kBlock) void temp_map_kernel(TempArgs a)
{
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= a.n) return;
    const float T = a.T[j];
    const float sg = a.sigma_max * fmaxf(0.0f, (T - a.soot_t0) / a.soot_span);
    if (a.em)
        for (int c = 0; c < 3; ++c) a.em[c * a.n + j] = lut_lookup(a.lut + c * a.lut_cap, a.lut_size, T, a.t_min, a.t_max);
    if (a.sig) a.sig[j] = sg;
    if (a.vol) {
        const float e = lut_lookup(a.lut + a.fit_channel * a.lut_cap, a.lut_size, T, a.t_min, a.t_max);
        reinterpret_cast<float2 *>(a.vol)[j] = make_float2(e, sg);
    }
}

__global__ __launch_bounds__(kBlock) void temp_invert_kernel(const float *e, float *T, const float *row,
                                                            int L, float t_min, float t_max, int64_t n)
{
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= n) return;
    const float x = fminf(fmaxf(e[j], row[0]), row[L - 1]);
    T[j] = lut_invert(row, L, x, t_min, t_max);
}

// Flame pixels (Sec. 4.1): 1 where any channel of the frame exceeds the threshold.
__global__ __launch_bounds__(kBlock) void flame_mask_kernel(const float *frames, int C, int V, int HW, float thr,
                                                           float *mask)
{
    const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (r >= (int64_t)V * HW) return;
    const int v = (int)(r / HW), pix = (int)(r - (int64_t)v * HW);
    float m = 0.0f;
    for (int c = 0; c < C; ++c)
        if (frames[((int64_t)v * C + c) * HW + pix] > thr) m = 1.0f;
    mask[r] = m;
}

// Visual hull (Alg. 1): a key point is inside when the eight cells around it
// carry, together, the flame-ray bits of every view.
__global__ __launch_bounds__(kBlock) void hull_assemble_kernel(const float *part, int ncells, int nx, int ny, int nz,
                                                              int bx, int by, uint64_t all, int32_t *inside,
                                                              int64_t n)
{
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= n) return;
    const int jx = (int)(j % nx), jy = (int)((j / nx) % ny), jz = (int)(j / ((int64_t)nx * ny));
    uint64_t bits = 0;
    for (int e = 0; e < 8; ++e) {
        const int cx = jx - (e & 1), cy = jy - ((e >> 1) & 1), cz = jz - ((e >> 2) & 1);
        if (cx < 0 || cy < 0 || cz < 0 || cx > nx - 2 || cy > ny - 2 || cz > nz - 2) continue;
        const int brick = ((cz >> 2) * by + (cy >> 3)) * bx + (cx >> 3);
        const int cell = brick * kBlock + (((cz & 3) * 8 + (cy & 7)) * 8 + (cx & 7));
        bits |= (uint64_t)__float_as_uint(part[cell]) | ((uint64_t)__float_as_uint(part[(int64_t)ncells + cell]) << 32);
    }
    inside[j] = bits == all ? 1 : 0;
}

// Key points outside the hull take a fixed value in every emission channel.
template <int C>
__global__ __launch_bounds__(kBlock) void apply_outside_kernel(float *vol, const int32_t *inside, float value, int64_t n)
{
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= n || inside[j]) return;
    if constexpr (C == 3) {
        float4 *p = reinterpret_cast<float4 *>(vol) + j;
        p->x = value;
        p->y = value;
        p->z = value;
    } else {
        reinterpret_cast<float2 *>(vol)[j].x = value;
    }
}

// Sum of the per-tile (squared residual, count) pairs in a fixed order, in
// double precision: one block, strided partial sums, then a fixed tree.
__global__ __launch_bounds__(kBlock) void err_reduce_kernel(const float2 *err, int n, double *out)
{
    __shared__ double s0[kBlock], s1[kBlock];
    double a0 = 0.0, a1 = 0.0;
    for (int i = threadIdx.x; i < n; i += kBlock) {
        a0 += (double)err[i].x;
        a1 += (double)err[i].y;
    }
    s0[threadIdx.x] = a0;
    s1[threadIdx.x] = a1;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            s0[threadIdx.x] += s0[threadIdx.x + w];
            s1[threadIdx.x] += s1[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = s0[0];
        out[1] = s1[0];
    }
}

static inline int blocks_for(int64_t n) { return (int)((n + kBlock - 1) / kBlock); }

// Cameras of a plan-free render, passed by value in the kernel arguments
// (nothing is copied from host memory at run time) and stored for the ray
// table kernel.
struct StaticCams {
    rte_camera cam[kStaticMaxViews];
    int n;
};

__global__ __launch_bounds__(64) void cams_store_kernel(StaticCams c, rte_camera *out)
{
    const int i = threadIdx.x;
    if (i < c.n) out[i] = c.cam[i];
}

// Launch order of a plan-free render: every tile in index order.
__global__ __launch_bounds__(kBlock) void iota_kernel(int32_t *out, int n)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) out[i] = i;
}

}  // namespace

// ------------------------------------------------------------ host launches

hipError_t launch_ray_table(const rte_plan *p, hipStream_t s)
{
    RayArgs a{};
    a.cams = p->d_cams;
    a.rayA = p->d_rayA;
    a.rayB = p->d_rayB;
    a.tnear = p->d_tnear;
    a.W = p->W;
    a.H = p->H;
    a.V = p->V;
    for (int i = 0; i < 3; ++i) {
        a.lo[i] = p->grid.bbox_min[i];
        a.hi[i] = p->grid.bbox_max[i];
        a.h[i] = p->h[i];
    }
    a.ds = p->ds;
    hipLaunchKernelGGL(ray_table_kernel, dim3(blocks_for(p->n_rays)), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_tile_kmax(const rte_plan *p, hipStream_t s)
{
    TileArgs a{p->d_rayB, p->d_tile_kmax, p->W, p->H, p->tiles_x, p->tiles_per_view, p->n_tiles};
    hipLaunchKernelGGL(tile_kmax_kernel, dim3(p->n_tiles), dim3(kTileRays), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_ray_export(const rte_plan *p, float *t_near, float *t_far, int32_t *nseg,
                             hipStream_t s)
{
    ExportArgs a{p->d_rayA, p->d_rayB, p->d_tnear, t_near, t_far, nseg, p->n_rays};
    hipLaunchKernelGGL(ray_export_kernel, dim3(blocks_for(p->n_rays)), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_pack(const rte_plan *p, const float *emission, const float *extinction,
                       int channels, hipStream_t s, bool keep_emission)
{
    PackArgs a{emission, extinction, p->d_vol, p->n_nodes, keep_emission ? 1 : 0};
    if (channels == 3)
        hipLaunchKernelGGL(pack_kernel<3>, dim3(blocks_for(p->n_nodes)), dim3(kBlock), 0, s, a);
    else
        hipLaunchKernelGGL(pack_kernel<1>, dim3(blocks_for(p->n_nodes)), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

// Planar residuals [V][3][H][W] -> one float4 (RGB, 0) per ray, the layout
// the gather reads.
__global__ __launch_bounds__(kBlock) void pack_residual_kernel(const float *planar, float4 *out, int V, int HW)
{
    const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (r >= (int64_t)V * HW) return;
    const int64_t v = r / HW, pix = r - v * HW;
    const float *p = planar + v * 3 * HW + pix;
    out[r] = make_float4(p[0], p[HW], p[2 * HW], 0.0f);
}

hipError_t launch_pack_residual(const rte_plan *p, const float *planar, const float **packed, hipStream_t s)
{
    if (p->params.channels != 3) {  // one channel: the layouts agree
        *packed = planar;
        return hipSuccess;
    }
    const int64_t n = (int64_t)p->V * p->W * p->H;
    hipLaunchKernelGGL(pack_residual_kernel, dim3(blocks_for(n)), dim3(kBlock), 0, s, planar,
                       reinterpret_cast<float4 *>(p->d_y), p->V, p->W * p->H);
    *packed = p->d_y;
    return hipGetLastError();
}

hipError_t launch_unpack(const rte_plan *p, float *emission, int channels, hipStream_t s)
{
    PackArgs a{nullptr, nullptr, p->d_vol, p->n_nodes, 0};
    if (channels == 3)
        hipLaunchKernelGGL(unpack_kernel<3>, dim3(blocks_for(p->n_nodes)), dim3(kBlock), 0, s, a, emission);
    else
        hipLaunchKernelGGL(unpack_kernel<1>, dim3(blocks_for(p->n_nodes)), dim3(kBlock), 0, s, a, emission);
    return hipGetLastError();
}

// In-scatter grids: one shared grid (isotropic phase function) or one per
// view (anisotropic), M^3 float4 entries each.
static int scat_view_stride(const rte_plan *p)
{
    const int M = p->params.scatter_res;
    return (p->params.phase_g != 0.0f && M >= 2) ? M * M * M : 0;
}

hipError_t launch_pack_scatter(const rte_plan *p, const float *planar, hipStream_t s)
{
    // planar [grids][C][M^3] -> packed [grids][M^3] float4, one grid per view
    // for an anisotropic phase function
    const int64_t m3 = (int64_t)p->params.scatter_res * p->params.scatter_res * p->params.scatter_res;
    const int grids = scat_view_stride(p) ? p->V : 1;
    const int C = p->params.channels;
    for (int v = 0; v < grids; ++v)
        hipLaunchKernelGGL(pack_scatter_kernel, dim3(blocks_for(m3)), dim3(kBlock), 0, s,
                           planar + (int64_t)v * C * m3, p->d_scat + (int64_t)v * m3, C, m3);
    return hipGetLastError();
}

template <int C, bool EMIS, bool SCAT, bool WG, int EPI>
static void render_launch(const RenderArgs &a, hipStream_t s)
{
    if (a.nb8 > 0)
        hipLaunchKernelGGL((render_kernel<C, EMIS, SCAT, WG, EPI>), dim3(a.nb8), dim3(kBlock), 0, s, a);
}

template <int C>
static hipError_t render_dispatch(const RenderArgs &a, bool emis, bool scat, bool wg, int epi,
                                  hipStream_t s)
{
    if (!emis) {
        // weights only (transmittance and per-sample weights); no epilogue
        render_launch<C, false, false, true, -1>(a, s);
        return hipGetLastError();
    }
#define RTE_EPI(E)                                                                        \
    if (epi == E) {                                                                       \
        if (scat && wg) render_launch<C, true, true, true, E>(a, s);                      \
        else if (scat) render_launch<C, true, true, false, E>(a, s);                      \
        else if (wg) render_launch<C, true, false, true, E>(a, s);                        \
        else render_launch<C, true, false, false, E>(a, s);                               \
        return hipGetLastError();                                                         \
    }
    RTE_EPI(kEpiImage)
    RTE_EPI(kEpiSart)
    RTE_EPI(kEpiMlem)
    RTE_EPI(kEpiPaper)
#undef RTE_EPI
    return hipErrorInvalidValue;
}

static RenderArgs render_args(const rte_plan *p, int epilogue, const float *frames, int frame_channels,
                              int frame_channel0, float *out, double *exit_tau, const float *mask, float2 *err)
{
    RenderArgs a{};
    a.sub_n = 1;
    a.sub_s = 0;
    a.exit_tau = exit_tau;
    a.mask = mask;
    a.err = err;
    a.fC = frame_channels;
    a.fc0 = frame_channel0;
    a.rayA = p->d_rayA;
    a.rayB = p->d_rayB;
    a.tile_off = p->d_tile_off;
    a.vol = p->d_vol;
    a.scat = p->d_scat;
    a.scat_vstride = scat_view_stride(p);
    a.frames = frames;
    a.out = out;
    a.g = p->d_g;
    a.W = p->W;
    a.H = p->H;
    a.tiles_x = p->tiles_x;
    a.tiles_per_view = p->tiles_per_view;
    a.n_tiles = p->n_tiles;
    a.tile_order = p->d_tile_order;
    // an image needs every pixel (misses get the background); residuals and
    // weights are only ever read for rays that hold samples
    // (the image error of the stop rule also needs the pixels of empty tiles)
    a.n_launch = (epilogue == kEpiImage || err) ? p->n_slots : p->n_active_slots;
    a.nb8 = (a.n_launch + 3) / 4;
    a.nx = p->grid.nx;
    a.ny = p->grid.ny;
    a.nz = p->grid.nz;
    a.M = p->params.scatter_res;
    a.ds = (float)p->ds;
    a.albedo = p->params.albedo;
    a.background = p->params.background;
    const int n[3] = {p->grid.nx, p->grid.ny, p->grid.nz};
    for (int i = 0; i < 3; ++i)
        a.s_scale[i] = a.M >= 2 ? (float)((double)(a.M - 1) / (double)(n[i] - 1)) : 0.0f;
    return a;
}

hipError_t launch_render(const rte_plan *p, int channels, bool use_emission, bool use_scatter,
                         bool write_g, int epilogue, const float *frames, int frame_channels,
                         int frame_channel0, float *out, hipStream_t s, double *exit_tau, const float *mask,
                         float2 *err, int sub_n, int sub_s)
{
    RenderArgs a = render_args(p, epilogue, frames, frame_channels, frame_channel0, out, exit_tau, mask, err);
    a.sub_n = sub_n;
    a.sub_s = sub_s;
    if (channels == 3) return render_dispatch<3>(a, use_emission, use_scatter, write_g, epilogue, s);
    return render_dispatch<1>(a, use_emission, use_scatter, write_g, epilogue, s);
}

// Arguments of a plan's in-scatter launches (every pass, and the reduce).
static ScatArgs scat_args(const rte_plan *p, float *planar_out)
{
    ScatArgs a{};
    a.vol = p->d_vol;
    a.dirs = p->d_dirs;
    a.dpart = p->d_scat_part;
    a.scat = p->d_scat;
    a.planar = planar_out;
    a.nx = p->grid.nx;
    a.ny = p->grid.ny;
    a.nz = p->grid.nz;
    a.M = p->params.scatter_res;
    a.ndirs = p->params.scatter_dirs;
    const int n[3] = {p->grid.nx, p->grid.ny, p->grid.nz};
    double hs_min = 1e300;
    for (int i = 0; i < 3; ++i) {
        a.p_scale[i] = (float)((double)(n[i] - 1) / (double)(a.M - 1));
        const double hs = (p->grid.bbox_max[i] - p->grid.bbox_min[i]) / (double)(a.M - 1);
        hs_min = hs < hs_min ? hs : hs_min;
    }
    a.ds = (float)(p->params.scatter_step * hs_min);
    a.inv_ndirs = 1.0f / (float)a.ndirs;
    const int bm = (a.M + 3) / 4;
    a.nbricks = bm * bm * bm;
    a.blocks_per_dir = (a.nbricks + 3) / 4;
    a.dirs_per_xcd = (a.ndirs + 7) / 8;
    const int64_t m3 = (int64_t)a.M * a.M * a.M;
    const int C = p->params.channels;
    a.kstate = reinterpret_cast<int *>(a.dpart + (int64_t)a.ndirs * C * m3);
    a.tstate = a.dpart + (int64_t)a.ndirs * (C + 1) * m3;
    const int64_t plane = (int64_t)a.nx * a.ny * (C == 3 ? 16 : 8);
    // a volume larger than one slab: XCD x owns slab x of 8, so each XCD's
    // L2 holds only its slab; a smaller volume is marched in one pass
    a.xslab = plane * (a.nz - 1) > kScatSlabBytes ? 1 : 0;
    a.nup = p->scat_nup;
    if (a.xslab) {
        a.npass = 8;
        a.slab_h = (float)((double)(a.nz - 1) / (double)a.npass);
        // brick layers (4 node planes each) of the nodes starting in each
        // slab, widened by one layer each side (the kernel checks each node)
        const int bmz = (a.M + 3) / 4;
        for (int sl = 0; sl < 8; ++sl) {
            a.bz_lo[sl] = bmz;
            a.bz_hi[sl] = -1;
        }
        for (int mz = 0; mz < a.M; ++mz) {
            const float pz = (float)mz * a.p_scale[2];
            const int sl = std::min(a.npass - 1, (int)(pz / a.slab_h));
            a.bz_lo[sl] = std::min(a.bz_lo[sl], mz / 4);
            a.bz_hi[sl] = std::max(a.bz_hi[sl], mz / 4);
        }
        for (int sl = 0; sl < 8; ++sl)
            if (a.bz_hi[sl] >= 0) {
                a.bz_lo[sl] = std::max(0, a.bz_lo[sl] - 1);
                a.bz_hi[sl] = std::min(bmz - 1, a.bz_hi[sl] + 1);
            }
    } else {
        a.npass = 1;
        a.slab_h = (float)(a.nz - 1);
    }
    const bool phase = scat_view_stride(p) != 0;
    if (phase) {
        a.cams = p->d_cams;
        a.dirs_world = p->d_dirs_world;
        a.V = p->V;
        a.phase_g = (double)p->params.phase_g;
        for (int i = 0; i < 3; ++i) {
            a.lo[i] = p->grid.bbox_min[i];
            a.hs[i] = (p->grid.bbox_max[i] - p->grid.bbox_min[i]) / (double)(a.M - 1);
        }
    }
    return a;
}

static int scat_passes(const ScatArgs &a) { return a.xslab ? kScatFinalPass + 1 : a.npass; }

// Blocks of march pass `pass` (0: nothing to march in it).
static int scat_pass_blocks(const ScatArgs &a, int pass)
{
    if (!a.xslab) return 8 * a.dirs_per_xcd * a.blocks_per_dir;
    // blocks per XCD: its up and down (direction, brick) items, 4 per block
    const int bxy = ((a.M + 3) / 4) * ((a.M + 3) / 4);
    int64_t most = 0;
    for (int xx = 0; xx < 8; ++xx) {
        const int su = xx - pass, sd = xx + pass;
        const int64_t nu = su >= 0 ? std::max(a.bz_hi[su] - a.bz_lo[su] + 1, 0) : 0;
        const int64_t ndn = sd < a.npass ? std::max(a.bz_hi[sd] - a.bz_lo[sd] + 1, 0) : 0;
        const int64_t items = (int64_t)a.nup * nu * bxy + (int64_t)(a.ndirs - a.nup) * ndn * bxy;
        most = std::max(most, (items + 3) / 4);
    }
    return (int)(8 * most);
}

hipError_t launch_inscatter(const rte_plan *p, float *planar_out, hipStream_t s)
{
    ScatArgs a = scat_args(p, planar_out);
    const int C = p->params.channels;
    const int64_t m3 = (int64_t)a.M * a.M * a.M;
    const bool phase = scat_view_stride(p) != 0;
    const dim3 rgrid((unsigned)blocks_for(m3), phase ? (unsigned)p->V : 1u);
    const dim3 sgrid((unsigned)((m3 + kReduceBlock - 1) / kReduceBlock));
    for (a.pass = 0; a.pass < scat_passes(a); ++a.pass) {
        const int nbp = scat_pass_blocks(a, a.pass);
        if (nbp == 0) continue;
        if (C == 3) hipLaunchKernelGGL(inscatter_march_kernel<3>, dim3(nbp), dim3(kBlock), 0, s, a);
        else hipLaunchKernelGGL(inscatter_march_kernel<1>, dim3(nbp), dim3(kBlock), 0, s, a);
    }
    if (C == 3) {
        if (phase) hipLaunchKernelGGL(inscatter_phase_reduce_kernel<3>, rgrid, dim3(kBlock), 0, s, a);
        else hipLaunchKernelGGL(inscatter_reduce_kernel<3>, sgrid, dim3(kReduceBlock), 0, s, a);
    } else {
        if (phase) hipLaunchKernelGGL(inscatter_phase_reduce_kernel<1>, rgrid, dim3(kBlock), 0, s, a);
        else hipLaunchKernelGGL(inscatter_reduce_kernel<1>, sgrid, dim3(kReduceBlock), 0, s, a);
    }
    return hipGetLastError();
}

// The in-scatter grids of n plans (one channel count) with one launch per
// march pass and one per kind of reduce, each covering every plan; the
// arguments and block-prefix tables go through plans[0]'s in-scatter
// staging region. Each plan's blocks do exactly what they do in its own
// launches (same pass, same XCD), so each grid is bitwise its own result.
hipError_t launch_inscatter_batch(rte_plan *const *plans, int n, hipStream_t s)
{
    constexpr int kMaxPass = kScatFinalPass + 1;
    std::vector<ScatArgs> sa(n);
    // prefix tables: one per march pass, then the isotropic and the per-view reduce
    std::vector<int> pre((size_t)(kMaxPass + 2) * (n + 1), 0);
    int npass = 0;
    for (int i = 0; i < n; ++i) {
        sa[i] = scat_args(plans[i], nullptr);
        npass = std::max(npass, scat_passes(sa[i]));
    }
    for (int t = 0; t < kMaxPass + 2; ++t) {
        int *pt = pre.data() + (size_t)t * (n + 1);
        for (int i = 0; i < n; ++i) {
            const ScatArgs &a = sa[i];
            const int64_t m3 = (int64_t)a.M * a.M * a.M;
            const bool phase = scat_view_stride(plans[i]) != 0;
            int nb = 0;
            if (t < kMaxPass) nb = t < scat_passes(a) ? scat_pass_blocks(a, t) : 0;
            else if (t == kMaxPass) nb = phase ? 0 : (int)((m3 + kReduceBlock - 1) / kReduceBlock);
            else nb = phase ? blocks_for(m3) * plans[i]->V : 0;
            pt[i + 1] = pt[i] + nb;  // march block counts are multiples of 8
        }
    }
    rte_plan *p0 = plans[0];
    const size_t o_a = p0->scat_stage_off, o_p = (o_a + sizeof(ScatArgs) * n + 15) & ~(size_t)15;
    const size_t bytes = o_p + sizeof(int) * pre.size() - o_a;
    if (o_a + bytes > p0->scat_stage_off + p0->scat_stage_bytes) return hipErrorInvalidValue;
    // the pinned region is rewritten only after its previous upload ended
    hipError_t e = hipEventSynchronize(p0->scat_event);
    if (e != hipSuccess) return e;
    char *h = static_cast<char *>(p0->h_batch);
    std::memcpy(h + o_a, sa.data(), sizeof(ScatArgs) * n);
    std::memcpy(h + o_p, pre.data(), sizeof(int) * pre.size());
    char *d = static_cast<char *>(p0->d_batch);
    e = hipMemcpyAsync(d + o_a, h + o_a, bytes, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    e = hipEventRecord(p0->scat_event, s);
    if (e != hipSuccess) return e;
    const ScatArgs *dsa = reinterpret_cast<const ScatArgs *>(d + o_a);
    const int *dpre = reinterpret_cast<const int *>(d + o_p);
    const int C = p0->params.channels;
    for (int t = 0; t < kMaxPass + 2; ++t) {
        const int total = pre[(size_t)t * (n + 1) + n];
        if (total == 0) continue;
        const int *pt = dpre + (size_t)t * (n + 1);
        if (t < kMaxPass) {
            if (C == 3) hipLaunchKernelGGL(inscatter_march_batch_kernel<3>, dim3(total), dim3(kBlock), 0, s, dsa, pt, n, t);
            else hipLaunchKernelGGL(inscatter_march_batch_kernel<1>, dim3(total), dim3(kBlock), 0, s, dsa, pt, n, t);
        } else if (t == kMaxPass) {
            if (C == 3) hipLaunchKernelGGL(inscatter_reduce_batch_kernel<3>, dim3(total), dim3(kReduceBlock), 0, s, dsa, pt, n);
            else hipLaunchKernelGGL(inscatter_reduce_batch_kernel<1>, dim3(total), dim3(kReduceBlock), 0, s, dsa, pt, n);
        } else {
            if (C == 3) hipLaunchKernelGGL(inscatter_phase_reduce_batch_kernel<3>, dim3(total), dim3(kBlock), 0, s, dsa, pt, n);
            else hipLaunchKernelGGL(inscatter_phase_reduce_batch_kernel<1>, dim3(total), dim3(kBlock), 0, s, dsa, pt, n);
        }
    }
    return hipGetLastError();
}

hipError_t launch_adjoint_march(const rte_plan *p, bool use_scatter, const double *exit_tau, const float *dI,
                                hipStream_t s)
{
    GradArgs a{};
    a.rayA = p->d_rayA;
    a.rayB = p->d_rayB;
    a.tile_off = p->d_tile_off;
    a.tile_order = p->d_tile_order;
    a.n_launch = p->n_active_slots;
    a.vol = p->d_vol;
    a.scat = p->d_scat;
    a.scat_vstride = scat_view_stride(p);
    a.exit_tau = exit_tau;
    a.dI = dI;
    a.gq = reinterpret_cast<float2 *>(p->d_q);
    a.W = p->W;
    a.H = p->H;
    a.tiles_x = p->tiles_x;
    a.tiles_per_view = p->tiles_per_view;
    a.nx = p->grid.nx;
    a.ny = p->grid.ny;
    a.nz = p->grid.nz;
    a.M = p->params.scatter_res;
    a.ds = (float)p->ds;
    a.albedo = p->params.albedo;
    a.background = p->params.background;
    const int n[3] = {p->grid.nx, p->grid.ny, p->grid.nz};
    for (int i = 0; i < 3; ++i)
        a.s_scale[i] = a.M >= 2 ? (float)((double)(a.M - 1) / (double)(n[i] - 1)) : 0.0f;
    const int nb = (a.n_launch + 3) / 4;
    if (nb == 0) return hipSuccess;
    const int C = p->params.channels;
    if (C == 3 && use_scatter) hipLaunchKernelGGL((adjoint_march_kernel<3, true>), dim3(nb), dim3(kBlock), 0, s, a);
    else if (C == 3) hipLaunchKernelGGL((adjoint_march_kernel<3, false>), dim3(nb), dim3(kBlock), 0, s, a);
    else if (use_scatter) hipLaunchKernelGGL((adjoint_march_kernel<1, true>), dim3(nb), dim3(kBlock), 0, s, a);
    else hipLaunchKernelGGL((adjoint_march_kernel<1, false>), dim3(nb), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

template <int C, int MODE>
static void gather_launch(const GatherArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL((gather_kernel<C, MODE>), dim3(a.nb8), dim3(kBlock), 0, s, a);
}

static GatherArgs gather_args(const rte_plan *p, const float *y, float alpha_l, float alpha_d, float tau,
                              const float *rowmask, float g_sigma, uint64_t seed, int iteration)
{
    GatherArgs a{};
    a.view0 = 0;
    a.view_step = 1;
    a.rowmask = rowmask;
    a.g_sigma = g_sigma;
    a.seed_lo = (uint32_t)seed;
    a.seed_hi = (uint32_t)(seed >> 32);
    a.iteration = iteration;
    a.rayA = p->d_rayA;
    a.rayB = p->d_rayB;
    a.tile_off = p->d_tile_off;
    a.g = p->d_g;
    a.q = p->d_q;
    a.y = y;
    a.proj = p->d_proj;
    a.part = p->d_part;
    a.V = p->V;
    a.W = p->W;
    a.H = p->H;
    a.tiles_x = p->tiles_x;
    a.tiles_per_view = p->tiles_per_view;
    a.nx = p->grid.nx;
    a.ny = p->grid.ny;
    a.nz = p->grid.nz;
    a.bx = (a.nx - 1 + 7) / 8;
    a.by = (a.ny - 1 + 7) / 8;
    a.bz = (a.nz - 1 + 3) / 4;
    a.nb8 = grid8((int64_t)a.bx * a.by * a.bz);
    a.ncells = (int)p->n_part_cells;
    a.ds = (float)p->ds;
    a.inv_ds = (float)(1.0 / p->ds);
    a.alpha_l = alpha_l;
    a.alpha_d = alpha_d;
    a.log2_keep = (float)std::log2(1.0 - (double)tau);
    return a;
}

hipError_t launch_gather(const rte_plan *p, int channels, int mode, const float *y, float alpha_l,
                         float alpha_d, float tau, hipStream_t s, const float *rowmask, float g_sigma,
                         uint64_t seed, int iteration, int view0, int view_step)
{
    if (view_step < 1 || view0 < 0) return hipErrorInvalidValue;
    // accumulators per corner this mode writes must fit the partial buffer
    const int need = mode == kGatherHull ? 2
                     : ((mode == kGatherAdjointCols || mode == kGatherGrad) ? channels + 1 : channels);
    if (need > p->part_acc) return hipErrorInvalidValue;
    GatherArgs a = gather_args(p, y, alpha_l, alpha_d, tau, rowmask, g_sigma, seed, iteration);
    a.view0 = view0;
    a.view_step = view_step;
    if (channels == 3) {
        switch (mode) {
        case kGatherAdjoint: gather_launch<3, kGatherAdjoint>(a, s); break;
        case kGatherAdjointCols: gather_launch<3, kGatherAdjointCols>(a, s); break;
        case kGatherPaper: gather_launch<3, kGatherPaper>(a, s); break;
        case kGatherGrad: gather_launch<3, kGatherGrad>(a, s); break;
        case kGatherHull: gather_launch<3, kGatherHull>(a, s); break;
        default: return hipErrorInvalidValue;
        }
    } else {
        switch (mode) {
        case kGatherAdjoint: gather_launch<1, kGatherAdjoint>(a, s); break;
        case kGatherAdjointCols: gather_launch<1, kGatherAdjointCols>(a, s); break;
        case kGatherPaper: gather_launch<1, kGatherPaper>(a, s); break;
        case kGatherGrad: gather_launch<1, kGatherGrad>(a, s); break;
        case kGatherHull: gather_launch<1, kGatherHull>(a, s); break;
        default: return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

template <int C, int MODE>
static void update_launch(const UpdateArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL((update_kernel<C, MODE>), dim3(grid8(a.nblocks)), dim3(kBlock), 0, s, a);
}

static UpdateArgs update_args(const rte_plan *p, int acc, float lambda, int clamp_nonneg, float *out,
                              float *temperature, int lut_size, int fit_channel, float *out2, const int32_t *inside)
{
    UpdateArgs a{};
    a.out2 = out2;
    a.inside = inside;
    a.part = p->d_part;
    a.vol = p->d_vol;
    a.cols = p->d_cols;
    a.out = out;
    a.temperature = temperature;
    a.lut = p->d_lut;
    a.lut_cap = p->lut_cap;
    a.lut_size = lut_size;
    a.fit_channel = fit_channel;
    a.t_min = p->lut_params.t_min;
    a.t_max = p->lut_params.t_max;
    a.nx = p->grid.nx;
    a.ny = p->grid.ny;
    a.nz = p->grid.nz;
    a.bx = (p->grid.nx - 1 + 7) / 8;
    a.by = (p->grid.ny - 1 + 7) / 8;
    a.bz = (p->grid.nz - 1 + 3) / 4;
    a.acc = acc;
    a.nbx = (p->grid.nx + 7) / 8;
    a.nby = (p->grid.ny + 7) / 8;
    a.nblocks = a.nbx * a.nby * ((p->grid.nz + 3) / 4);
    a.n = p->n_nodes;
    a.lambda = lambda;
    a.clamp_nonneg = clamp_nonneg;
    return a;
}

hipError_t launch_update(const rte_plan *p, int channels, int acc, int mode, float lambda,
                         int clamp_nonneg, float *out, float *temperature, int lut_size,
                         int fit_channel, hipStream_t s, float *out2, const int32_t *inside, float *cols_out)
{
    UpdateArgs a =
        update_args(p, acc, lambda, clamp_nonneg, out, temperature, lut_size, fit_channel, out2, inside);
    a.cols_out = cols_out;
#define RTE_UPD(M)                                            \
    case M:                                                   \
        if (channels == 3) update_launch<3, M>(a, s);         \
        else update_launch<1, M>(a, s);                       \
        break;
    switch (mode) {
        RTE_UPD(kUpdDelta)
        RTE_UPD(kUpdSart)
        RTE_UPD(kUpdMlem)
        RTE_UPD(kUpdPaper)
        RTE_UPD(kUpdGrad)
        RTE_UPD(kUpdSartOS)
        RTE_UPD(kUpdMlemOS)
    case kUpdTemp: update_launch<1, kUpdTemp>(a, s); break;
    default: return hipErrorInvalidValue;
    }
#undef RTE_UPD
    return hipGetLastError();
}

hipError_t launch_temp_map(const rte_plan *p, const float *T, float *em_planar, float *sig_planar,
                           bool packed, int lut_size, int fit_channel, float sigma_max,
                           float soot_t0, float soot_span, float t_min, float t_max, hipStream_t s)
{
    TempArgs a{};
    a.T = T;
    a.lut = p->d_lut;
    a.em = em_planar;
    a.sig = sig_planar;
    a.vol = packed ? p->d_vol : nullptr;
    a.lut_cap = p->lut_cap;
    a.lut_size = lut_size;
    a.fit_channel = fit_channel;
    a.t_min = t_min;
    a.t_max = t_max;
    a.sigma_max = sigma_max;
    a.soot_t0 = soot_t0;
    a.soot_span = soot_span;
    a.n = p->n_nodes;
    hipLaunchKernelGGL(temp_map_kernel, dim3(blocks_for(a.n)), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_temp_invert(const rte_plan *p, const float *e, float *T, int lut_size,
                              int fit_channel, float t_min, float t_max, hipStream_t s)
{
    hipLaunchKernelGGL(temp_invert_kernel, dim3(blocks_for(p->n_nodes)), dim3(kBlock), 0, s, e, T,
                       p->d_lut + (size_t)fit_channel * p->lut_cap, lut_size, t_min, t_max,
                       p->n_nodes);
    return hipGetLastError();
}

hipError_t launch_flame_mask(const rte_plan *p, const float *frames, int frame_channels, float threshold,
                             float *mask, hipStream_t s)
{
    hipLaunchKernelGGL(flame_mask_kernel, dim3(blocks_for(p->n_rays)), dim3(kBlock), 0, s, frames, frame_channels,
                       p->V, p->W * p->H, threshold, mask);
    return hipGetLastError();
}

hipError_t launch_hull(const rte_plan *p, const float *mask, int32_t *inside, hipStream_t s)
{
    hipError_t e = launch_gather(p, 1, kGatherHull, nullptr, 0.f, 0.f, 0.f, s, mask, 0.f, 0, 0);
    if (e != hipSuccess) return e;
    const uint64_t all = p->V == 64 ? ~(uint64_t)0 : (((uint64_t)1 << p->V) - 1);
    hipLaunchKernelGGL(hull_assemble_kernel, dim3(blocks_for(p->n_nodes)), dim3(kBlock), 0, s, p->d_part,
                       (int)p->n_part_cells, p->grid.nx, p->grid.ny, p->grid.nz, (p->grid.nx - 1 + 7) / 8,
                       (p->grid.ny - 1 + 7) / 8, all, inside, p->n_nodes);
    return hipGetLastError();
}

hipError_t launch_apply_outside(const rte_plan *p, int channels, const int32_t *inside, float value, hipStream_t s)
{
    if (channels == 3)
        hipLaunchKernelGGL(apply_outside_kernel<3>, dim3(blocks_for(p->n_nodes)), dim3(kBlock), 0, s, p->d_vol, inside,
                           value, p->n_nodes);
    else
        hipLaunchKernelGGL(apply_outside_kernel<1>, dim3(blocks_for(p->n_nodes)), dim3(kBlock), 0, s, p->d_vol, inside,
                           value, p->n_nodes);
    return hipGetLastError();
}

hipError_t launch_err_reduce(const rte_plan *p, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(err_reduce_kernel, dim3(1), dim3(kBlock), 0, s, p->d_err, p->n_slots, out);
    return hipGetLastError();
}

// One reconstruction iteration for n plans with open jobs: one launch per
// phase (render with residual, voxel-owned gather, update) covering every
// plan's tiles, bricks and key points. The per-plan arguments and the block
// prefix tables are staged in plans[0]'s batch buffer.
template <int C, int EPI, int GMODE, int UMODE>
static hipError_t step_batch(rte_plan *const *plans, int n, bool scat, hipStream_t s, hipEvent_t *marks)
{
    std::vector<RenderArgs> ra(n);
    std::vector<GatherArgs> ga(n);
    std::vector<UpdateArgs> ua(n);
    std::vector<int> rp(n + 1, 0), gp(n + 1, 0), up(n + 1, 0);
    for (int i = 0; i < n; ++i) {
        const rte_plan *p = plans[i];
        const rte_recon_params &q = p->job_params;
        ra[i] = render_args(p, EPI, p->job_frames, C, 0, p->d_y, nullptr, q.use_mask ? p->d_mask : nullptr, nullptr);
        ga[i] = gather_args(p, p->d_y, q.alpha_l, q.alpha_d, q.tau, nullptr, q.g_sigma, q.seed, p->job_iter);
        ua[i] = update_args(p, C, q.lambda, q.clamp_nonneg, nullptr, nullptr, 0, 0, nullptr,
                            q.use_hull ? p->d_inside : nullptr);
        // each plan's render blocks start on XCD 0, as when launched alone
        rp[i + 1] = rp[i] + grid8(ra[i].nb8);
        gp[i + 1] = gp[i] + ga[i].bx * ga[i].by * ga[i].bz;
        up[i + 1] = up[i] + ua[i].nblocks;
    }
    // staging layout: [render args][gather args][update args][3 prefix tables]
    char *d = static_cast<char *>(plans[0]->d_batch);
    const size_t o_r = 0, o_g = o_r + sizeof(RenderArgs) * n, o_u = o_g + sizeof(GatherArgs) * n;
    const size_t o_p = (o_u + sizeof(UpdateArgs) * n + 15) & ~(size_t)15;
    const size_t np = (size_t)(n + 1) * sizeof(int);
    if (o_p + 3 * np > plans[0]->batch_bytes) return hipErrorInvalidValue;
    // the pinned staging buffer is rewritten only after its previous upload ended
    hipError_t e = hipEventSynchronize(plans[0]->batch_event);
    if (e != hipSuccess) return e;
    char *h = static_cast<char *>(plans[0]->h_batch);
    std::memcpy(h + o_r, ra.data(), sizeof(RenderArgs) * n);
    std::memcpy(h + o_g, ga.data(), sizeof(GatherArgs) * n);
    std::memcpy(h + o_u, ua.data(), sizeof(UpdateArgs) * n);
    std::memcpy(h + o_p, rp.data(), np);
    std::memcpy(h + o_p + np, gp.data(), np);
    std::memcpy(h + o_p + 2 * np, up.data(), np);
    e = hipMemcpyAsync(d, h, o_p + 3 * np, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    e = hipEventRecord(plans[0]->batch_event, s);
    if (e != hipSuccess) return e;
    const RenderArgs *dra = reinterpret_cast<const RenderArgs *>(d + o_r);
    const GatherArgs *dga = reinterpret_cast<const GatherArgs *>(d + o_g);
    const UpdateArgs *dua = reinterpret_cast<const UpdateArgs *>(d + o_u);
    const int *drp = reinterpret_cast<const int *>(d + o_p), *dgp = reinterpret_cast<const int *>(d + o_p + np),
              *dup = reinterpret_cast<const int *>(d + o_p + 2 * np);
    // marks (optional): start/stop events around the render, gather and update launches
    auto mark = [&](int i) { if (marks && marks[i]) (void)hipEventRecord(marks[i], s); };
    mark(0);
    if (rp[n] > 0) {
        if (scat)
            hipLaunchKernelGGL((render_batch_kernel<C, true, true, false, EPI>), dim3(rp[n]), dim3(kBlock), 0, s, dra, drp, n);
        else
            hipLaunchKernelGGL((render_batch_kernel<C, true, false, false, EPI>), dim3(rp[n]), dim3(kBlock), 0, s, dra, drp, n);
    }
    mark(1);
    mark(2);
    if (gp[n] > 0) hipLaunchKernelGGL((gather_batch_kernel<C, GMODE>), dim3(gp[n]), dim3(kBlock), 0, s, dga, dgp, n);
    mark(3);
    mark(4);
    if (up[n] > 0) hipLaunchKernelGGL((update_batch_kernel<C, UMODE>), dim3(grid8(up[n])), dim3(kBlock), 0, s, dua, dup, n, up[n]);
    mark(5);
    return hipGetLastError();
}

hipError_t launch_step_batch(rte_plan *const *plans, int n, hipStream_t s, hipEvent_t *marks)
{
    const int C = plans[0]->params.channels;
    const bool scat = plans[0]->params.albedo > 0.0f && plans[0]->params.scatter_res >= 2;
    const int upd = plans[0]->job_params.update;
#define RTE_STEP(CC)                                                                                   \
    if (upd == RTE_UPDATE_SART) return step_batch<CC, kEpiSart, kGatherAdjoint, kUpdSart>(plans, n, scat, s, marks); \
    if (upd == RTE_UPDATE_MLEM) return step_batch<CC, kEpiMlem, kGatherAdjoint, kUpdMlem>(plans, n, scat, s, marks); \
    return step_batch<CC, kEpiPaper, kGatherPaper, kUpdPaper>(plans, n, scat, s, marks);
    if (C == 3) { RTE_STEP(3) }
    RTE_STEP(1)
#undef RTE_STEP
}

}  // namespace rte

// ---------------------------------------------- render without a plan

// Workspace of rte_render_static: one array per GPU, held until the process
// ends. Host code never passes `scratch` itself to a kernel (on the host it is
// only a stand-in for the symbol): each device's address is looked up once
// with hipGetSymbolAddress and kernels receive that address.
static __device__ __align__(256) unsigned char scratch[rte::kStaticScratchBytes];

namespace rte {
namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_addr[kMaxDevices] = {};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

hipError_t static_scratch(void **addr)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_addr[dev] = p;
    }
    *addr = g_scratch_addr[dev];
    return hipSuccess;
}

StaticLayout static_layout(int V, int W, int H, int64_t n_nodes, int C, int M, bool per_view_scatter)
{
    StaticLayout L{};
    const int64_t rays = (int64_t)V * W * H;
    const int64_t tiles = (int64_t)V * ((W + kTile - 1) / kTile) * ((H + kTile - 1) / kTile);
    size_t at = 0;
    auto take = [&](size_t bytes) {
        const size_t here = at;
        at += align256(bytes);
        return here;
    };
    L.cams = take(sizeof(rte_camera) * (size_t)V);
    L.rayA = take(sizeof(float4) * (size_t)rays);
    L.rayB = take(sizeof(float4) * (size_t)rays);
    L.tnear = take(sizeof(float) * (size_t)rays);
    L.order = take(sizeof(int32_t) * (size_t)tiles);
    L.vol = take((C == 3 ? 16 : 8) * (size_t)n_nodes);
    const size_t grids = per_view_scatter ? (size_t)V : 1;
    L.scat = take(M >= 2 ? sizeof(float4) * grids * (size_t)M * M * M : 0);
    L.total = at;
    return L;
}

hipError_t launch_render_static(rte_plan *view, const rte_camera *cams, const float *emission,
                                const float *extinction, const float *inscatter, float *images, hipStream_t s)
{
    void *base = nullptr;
    hipError_t e = static_scratch(&base);
    if (e != hipSuccess) return e;
    unsigned char *b = static_cast<unsigned char *>(base);
    const rte_render_params &pr = view->params;
    const int C = pr.channels;
    const int M = pr.scatter_res >= 2 ? pr.scatter_res : 0;
    const StaticLayout L = static_layout(view->V, view->W, view->H, view->n_nodes, C, M, pr.phase_g != 0.0f);
    if (L.total > kStaticScratchBytes) return hipErrorOutOfMemory;
    if (view->V > kStaticMaxViews) return hipErrorInvalidValue;
    view->d_cams = reinterpret_cast<rte_camera *>(b + L.cams);
    view->d_rayA = reinterpret_cast<float4 *>(b + L.rayA);
    view->d_rayB = reinterpret_cast<float4 *>(b + L.rayB);
    view->d_tnear = reinterpret_cast<float *>(b + L.tnear);
    view->d_tile_order = reinterpret_cast<int32_t *>(b + L.order);
    view->d_vol = reinterpret_cast<float *>(b + L.vol);
    view->d_scat = M ? reinterpret_cast<float4 *>(b + L.scat) : nullptr;
    view->n_active_slots = view->n_slots = view->n_tiles;
    // every byte the render reads is written earlier in this call: nothing
    // in the array has to start at zero
    StaticCams sc{};
    for (int v = 0; v < view->V; ++v) sc.cam[v] = cams[v];
    sc.n = view->V;
    hipLaunchKernelGGL(cams_store_kernel, dim3(1), dim3(64), 0, s, sc, view->d_cams);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = launch_ray_table(view, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(iota_kernel, dim3(blocks_for(view->n_tiles)), dim3(kBlock), 0, s, view->d_tile_order,
                       view->n_tiles);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = launch_pack(view, emission, extinction, C, s)) != hipSuccess) return e;
    const bool scat = inscatter && pr.albedo > 0.0f && M;
    if (scat && (e = launch_pack_scatter(view, inscatter, s)) != hipSuccess) return e;
    return launch_render(view, C, true, scat, false, kEpiImage, nullptr, C, 0, images, s);
}

}  // namespace rte
