/*
 * rte_oracle.c -- plain, slow, FP64 CPU oracle for radiative-transport
 * flame volume reconstruction (Shen et al., "Radiative Transport Based
 * Flame Volume Reconstruction from Videos", arXiv:1809.06417).
 *
 * TEST INFRASTRUCTURE ONLY. The test-suite, the smoke check and the CPU
 * baseline leg of the benchmark are the only users of this library. It
 * shares no source, header, table or helper with the HIP library, and the
 * HIP library never loads it.
 *
 * Every function follows a passage of the paper; where the paper is silent
 * the reading used is stated next to the code. Arithmetic is double
 * precision throughout. Parallel loops (OpenMP) only split independent rays
 * or key points; every sum that crosses threads is reduced in a fixed
 * thread order, so results are reproducible for a given thread count.
 *
 * Conventions (shared with the callers, not with the GPU code):
 *  - Grid: n[a] key points per axis a (x, y, z) at the voxel vertices
 *    (Sec. 3.3, "Key points"), spanning [lo, hi]; fields are stored
 *    [z][y][x] with x fastest. h_a = (hi_a - lo_a) / (n_a - 1).
 *  - Camera: x_c = R x_w + t, pixel (u, v) centre at (u + 1/2, v + 1/2),
 *    u to the right, v downwards, optical axis +z_c (pinhole perspective
 *    projection, Sec. 3.2 and Sec. 4.1).
 *  - Images: [view][channel][v][u]. Volumes: [channel][z][y][x].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    double fx, fy, cx, cy;
    double R[9]; /* row-major world -> camera rotation */
    double t[3];
    int32_t width, height;
} orc_camera;

typedef struct {
    int32_t n[3]; /* key points along x, y, z */
    double lo[3], hi[3];
} orc_grid;

typedef struct {
    double t_min, t_max;  /* LUT domain [K] */
    double t_norm;        /* normalising temperature [K] */
    double band_nm[3];    /* camera band centres, R G B [nm] */
    double band_std_nm;   /* Gaussian band standard deviation [nm] */
    int32_t lut_size;
    double sigma_max;     /* extinction at full soot load [1/unit length] */
    double soot_t0;       /* soot appears above this temperature [K] */
    double soot_span;     /* soot load reaches 1 at soot_t0 + soot_span [K] */
    int32_t channel;      /* channel used for the fit (1 = green) */
    int32_t panels;       /* Simpson panels for each band integral */
} orc_temp_params;

#define ORC_MAX_THREADS 32

static int n_threads(void)
{
#ifdef _OPENMP
    int t = omp_get_max_threads();
    return t > ORC_MAX_THREADS ? ORC_MAX_THREADS : (t < 1 ? 1 : t);
#else
    return 1;
#endif
}

static int thread_id(void)
{
#ifdef _OPENMP
    return omp_get_thread_num();
#else
    return 0;
#endif
}

/* ---------------------------------------------------------------- grid */

static long grid_nodes(const orc_grid *g) { return (long)g->n[0] * g->n[1] * g->n[2]; }

static void grid_spacing(const orc_grid *g, double h[3])
{
    for (int a = 0; a < 3; ++a) h[a] = (g->hi[a] - g->lo[a]) / (double)(g->n[a] - 1);
}

static double grid_min_spacing(const orc_grid *g)
{
    double h[3];
    grid_spacing(g, h);
    double m = h[0];
    if (h[1] < m) m = h[1];
    if (h[2] < m) m = h[2];
    return m;
}

/* Trilinear stencil of a point (Sec. 3.3: a sample point touches its eight
 * neighbouring key points). q holds grid coordinates (units of h); they are
 * clamped to [0, n-1] and the cell index to n-2, so the stencil always has
 * eight valid corners. idx/w receive the corners in (dz, dy, dx) binary
 * order. */
static void stencil(const orc_grid *g, const double q[3], long idx[8], double w[8], double frac[3],
                    int cell[3])
{
    double f[3];
    int i[3];
    for (int a = 0; a < 3; ++a) {
        double c = q[a];
        double top = (double)(g->n[a] - 1);
        if (c < 0.0) c = 0.0;
        if (c > top) c = top;
        int ia = (int)floor(c);
        if (ia > g->n[a] - 2) ia = g->n[a] - 2;
        i[a] = ia;
        f[a] = c - (double)ia;
    }
    long nx = g->n[0], nxy = (long)g->n[0] * g->n[1];
    for (int corner = 0; corner < 8; ++corner) {
        int dx = corner & 1, dy = (corner >> 1) & 1, dz = (corner >> 2) & 1;
        idx[corner] = (long)(i[2] + dz) * nxy + (long)(i[1] + dy) * nx + (i[0] + dx);
        w[corner] = (dx ? f[0] : 1.0 - f[0]) * (dy ? f[1] : 1.0 - f[1]) * (dz ? f[2] : 1.0 - f[2]);
    }
    if (frac) for (int a = 0; a < 3; ++a) frac[a] = f[a];
    if (cell) for (int a = 0; a < 3; ++a) cell[a] = i[a];
}

static double trilerp(const orc_grid *g, const double *field, const double q[3])
{
    long idx[8];
    double w[8];
    stencil(g, q, idx, w, NULL, NULL);
    double s = 0.0;
    for (int c = 0; c < 8; ++c) s += w[c] * field[idx[c]];
    return s;
}

static void to_grid_coords(const orc_grid *g, const double p[3], double q[3])
{
    double h[3];
    grid_spacing(g, h);
    for (int a = 0; a < 3; ++a) q[a] = (p[a] - g->lo[a]) / h[a];
}

/* ------------------------------------------------------------- cameras */

/* Pinhole ray through the centre of pixel (u, v): origin at the camera
 * centre -R^T t, unit direction R^T K^{-1} (u + 1/2, v + 1/2, 1)^T. */
static void camera_ray(const orc_camera *c, int u, int v, double o[3], double d[3])
{
    double dc[3] = {((double)u + 0.5 - c->cx) / c->fx, ((double)v + 0.5 - c->cy) / c->fy, 1.0};
    double n2 = 0.0;
    for (int i = 0; i < 3; ++i) {
        d[i] = c->R[0 * 3 + i] * dc[0] + c->R[1 * 3 + i] * dc[1] + c->R[2 * 3 + i] * dc[2];
        o[i] = -(c->R[0 * 3 + i] * c->t[0] + c->R[1 * 3 + i] * c->t[1] + c->R[2 * 3 + i] * c->t[2]);
        n2 += d[i] * d[i];
    }
    double inv = 1.0 / sqrt(n2);
    for (int i = 0; i < 3; ++i) d[i] *= inv;
}

/* Entry/exit of the ray o + t d (t >= 0) through the box [lo, hi] (slab
 * method). Returns 1 when the ray crosses a segment of positive length. */
static int ray_box(const double lo[3], const double hi[3], const double o[3], const double d[3],
                   double *tn, double *tf)
{
    double t0 = -INFINITY, t1 = INFINITY;
    for (int a = 0; a < 3; ++a) {
        if (d[a] != 0.0) {
            double ta = (lo[a] - o[a]) / d[a], tb = (hi[a] - o[a]) / d[a];
            if (ta > tb) { double s = ta; ta = tb; tb = s; }
            if (ta > t0) t0 = ta;
            if (tb < t1) t1 = tb;
        } else if (o[a] < lo[a] || o[a] > hi[a]) {
            return 0;
        }
    }
    if (t0 < 0.0) t0 = 0.0;
    *tn = t0;
    *tf = t1;
    return t1 > t0;
}

/* Segments of a chord [tn, tf] with step ds (Sec. 4.2: samples spaced at a
 * fixed step along each ray). K = ceil((tf - tn) / ds); segment k spans
 * [tn + k ds, min(tn + (k+1) ds, tf)] and its sample sits at the midpoint,
 * so the last segment is clipped at the exit. */
static int n_segments(double tn, double tf, double ds)
{
    if (!(tf > tn)) return 0;
    return (int)ceil((tf - tn) / ds);
}

static void segment(double tn, double tf, double ds, int k, double *tmid, double *len)
{
    double a = tn + (double)k * ds;
    double b = tn + (double)(k + 1) * ds;
    if (b > tf) b = tf;
    if (b < a) b = a;
    *len = b - a;
    *tmid = 0.5 * (a + b);
}

/* phi(x) = (1 - e^{-x}) / x, phi(0) = 1: exact integral of the transmittance
 * over a segment of optical thickness x, divided by x. */
static double phi(double x)
{
    if (x == 0.0) return 1.0;
    return -expm1(-x) / x;
}

static int camera_index_ok(const orc_camera *c) { return c->width > 0 && c->height > 0; }

/* --------------------------------------------------------------- rays */

/* Ray table: entry distance, exit distance and number of segments of every
 * pixel ray, in [view][v][u] order. Misses get K = 0 and t_near = t_far = 0. */
int orc_ray_table(const orc_grid *g, const orc_camera *cams, int32_t V, double step_vox,
                  double *t_near, double *t_far, int32_t *K)
{
    double ds = step_vox * grid_min_spacing(g);
    for (int v = 0; v < V; ++v) {
        const orc_camera *c = &cams[v];
        if (!camera_index_ok(c)) return -1;
        long base = (long)v * c->width * c->height;
#pragma omp parallel for schedule(static)
        for (long p = 0; p < (long)c->width * c->height; ++p) {
            int u = (int)(p % c->width), vv = (int)(p / c->width);
            double o[3], d[3], tn, tf;
            camera_ray(c, u, vv, o, d);
            if (ray_box(g->lo, g->hi, o, d, &tn, &tf)) {
                t_near[base + p] = tn;
                t_far[base + p] = tf;
                K[base + p] = n_segments(tn, tf, ds);
            } else {
                t_near[base + p] = 0.0;
                t_far[base + p] = 0.0;
                K[base + p] = 0;
            }
        }
    }
    return 0;
}

/* ------------------------------------------------------------- render */

/* Emission-absorption(-in-scattering) render of every pixel of every view.
 *
 * Eq. 5 along one ray, with the optical model of Eq. 6, integrated exactly
 * for piecewise-constant extinction and source on each segment and composed
 * front to back as in Eq. 7-8 (segment opacity 1 - e^{-sigma Delta}, segment
 * radiance j / sigma):
 *   I_c = sum_k T_k j_kc Delta_k phi(sigma_k Delta_k) + T_K L_bg,
 *   T_{k+1} = T_k e^{-sigma_k Delta_k},  T_0 = 1,
 *   j_kc = eps_c(x_k) + albedo * sigma(x_k) * S_c(x_k),
 *   sigma(x) = max(0, trilinear extinction).
 * The emission field is the emitted colour intensity itself (Sec. 3.3,
 * "Emission"). S (in-scattered radiance, Eq. 5 third term) is a grid of
 * s_res^3 nodes over the same box, or NULL.
 *
 * em [C][N], sig [N], S [C][s_res^3] or NULL, img [V][C][H][W].
 * rowsum [V][H][W] (optional) receives sum_k T_k Delta_k phi_k. */
/* In-scatter grid seen by view v: one grid [C][M^3] shared by all views
 * (isotropic phase function), or grids [V][C][M^3], one per view
 * (anisotropic phase function, see orc_inscatter_phase). */
static const double *view_grid(const double *S, int s_views, int v, int C, int s_res)
{
    return s_views ? S + (long)v * C * s_res * s_res * s_res : S;
}

/* Render every view (Eq. 5-8 with the segment rule above). img [V][C][H][W];
 * rowsum (optional) [V][H][W] receives sum_k T_k Delta_k phi_k, the row sums
 * of the linear emission -> image map. S: in-scatter grid(s) as described at
 * view_grid, NULL without in-scattering. */
int orc_render(const orc_grid *g, const orc_camera *cams, int32_t V, int32_t C, double step_vox,
               double albedo, double background, const double *em, const double *sig,
               int32_t s_res, const double *S, int32_t s_views, double *img, double *rowsum)
{
    if (C < 1) return -1;
    double ds = step_vox * grid_min_spacing(g);
    long N = grid_nodes(g);
    orc_grid sg;
    if (S) {
        for (int a = 0; a < 3; ++a) { sg.n[a] = s_res; sg.lo[a] = g->lo[a]; sg.hi[a] = g->hi[a]; }
    }
    for (int v = 0; v < V; ++v) {
        const orc_camera *c = &cams[v];
        if (!camera_index_ok(c)) return -1;
        long HW = (long)c->width * c->height;
        const double *Sv = S ? view_grid(S, s_views, v, C, s_res) : NULL;
#pragma omp parallel for schedule(static)
        for (long p = 0; p < HW; ++p) {
            int u = (int)(p % c->width), vv = (int)(p / c->width);
            double o[3], d[3], tn, tf;
            double I[16];
            for (int ch = 0; ch < C; ++ch) I[ch] = 0.0;
            double T = 1.0, R = 0.0;
            camera_ray(c, u, vv, o, d);
            if (ray_box(g->lo, g->hi, o, d, &tn, &tf)) {
                int K = n_segments(tn, tf, ds);
                for (int k = 0; k < K; ++k) {
                    double t, len, x[3], q[3];
                    segment(tn, tf, ds, k, &t, &len);
                    for (int a = 0; a < 3; ++a) x[a] = o[a] + t * d[a];
                    to_grid_coords(g, x, q);
                    double s = trilerp(g, sig, q);
                    if (s < 0.0) s = 0.0;
                    double wgt = T * len * phi(s * len);
                    for (int ch = 0; ch < C; ++ch) {
                        double j = trilerp(g, em + (long)ch * N, q);
                        if (S && albedo != 0.0) {
                            double qs[3];
                            to_grid_coords(&sg, x, qs);
                            j += albedo * s * trilerp(&sg, Sv + (long)ch * s_res * s_res * s_res, qs);
                        }
                        I[ch] += wgt * j;
                    }
                    R += wgt;
                    T *= exp(-s * len);
                }
            }
            for (int ch = 0; ch < C; ++ch)
                img[((long)v * C + ch) * HW + p] = I[ch] + T * background;
            if (rowsum) rowsum[(long)v * HW + p] = R;
        }
    }
    return 0;
}

/* ---------------------------------------------------------- in-scatter */

/* Spherical Fibonacci direction d of n (unit vector). */
static void fib_dir(int d, int n, double u[3])
{
    double z = 1.0 - (2.0 * d + 1.0) / (double)n;
    double r = sqrt(fmax(0.0, 1.0 - z * z));
    double ph = (double)d * M_PI * (3.0 - sqrt(5.0));
    u[0] = r * cos(ph);
    u[1] = r * sin(ph);
    u[2] = z;
}

/* In-scattered radiance grid (Eq. 5 third term with the isotropic phase
 * function of Eq. 9 at g = 0, so the scattering integral is the mean
 * incident radiance). At each of the s_res^3 nodes p of a grid over the same
 * box:
 *   S_c(p) = (1/n_dirs) sum_d L_c(p <- u_d),
 *   L_c(p <- u) = emission-absorption march from p along u to the box exit,
 * with n_dirs spherical-Fibonacci directions, segments of
 * s_step * (coarse node spacing) and the same segment rule as the render.
 * Single scattering: the march uses the emission only. */
/* World position of in-scatter node (mx, my, mz): the M nodes per axis span
 * the closed bounding box, node M-1 on the upper face. lo + (M-1) h can land
 * an ulp past hi in FP64, which would put a face node outside the box and
 * drop the rays that run along that face; the node is clamped into the box. */
static void scat_node(const orc_grid *g, const double hs[3], int mx, int my, int mz, double p[3])
{
    const int m[3] = {mx, my, mz};
    for (int a = 0; a < 3; ++a) {
        const double v = g->lo[a] + m[a] * hs[a];
        p[a] = v < g->lo[a] ? g->lo[a] : (v > g->hi[a] ? g->hi[a] : v);
    }
}

int orc_inscatter(const orc_grid *g, int32_t C, const double *em, const double *sig, int32_t s_res,
                  int32_t n_dirs, double s_step, double *S)
{
    if (s_res < 2 || n_dirs < 1) return -1;
    long N = grid_nodes(g);
    orc_grid sg;
    for (int a = 0; a < 3; ++a) { sg.n[a] = s_res; sg.lo[a] = g->lo[a]; sg.hi[a] = g->hi[a]; }
    double hs[3];
    grid_spacing(&sg, hs);
    double ds = s_step * grid_min_spacing(&sg);
    long M3 = (long)s_res * s_res * s_res;
#pragma omp parallel for schedule(static)
    for (long m = 0; m < M3; ++m) {
        int mx = (int)(m % s_res), my = (int)((m / s_res) % s_res), mz = (int)(m / ((long)s_res * s_res));
        double p[3];
        scat_node(g, hs, mx, my, mz, p);
        double acc[16];
        for (int ch = 0; ch < C; ++ch) acc[ch] = 0.0;
        for (int dd = 0; dd < n_dirs; ++dd) {
            double u[3], tn, tf;
            fib_dir(dd, n_dirs, u);
            if (!ray_box(g->lo, g->hi, p, u, &tn, &tf)) continue;
            int K = n_segments(tn, tf, ds);
            double T = 1.0;
            for (int k = 0; k < K; ++k) {
                double t, len, x[3], q[3];
                segment(tn, tf, ds, k, &t, &len);
                for (int a = 0; a < 3; ++a) x[a] = p[a] + t * u[a];
                to_grid_coords(g, x, q);
                double s = trilerp(g, sig, q);
                if (s < 0.0) s = 0.0;
                double wgt = T * len * phi(s * len);
                for (int ch = 0; ch < C; ++ch) acc[ch] += wgt * trilerp(g, em + (long)ch * N, q);
                T *= exp(-s * len);
            }
        }
        for (int ch = 0; ch < C; ++ch) S[(long)ch * M3 + m] = acc[ch] / (double)n_dirs;
    }
    return 0;
}

/* Henyey-Greenstein phase function in the form of Eq. 9, p(w, w_i) with
 * w the direction of interest (the direction the scattered light travels)
 * and w_i the direction the incident light comes from (pointing from the
 * point towards its source). With the plus sign of Eq. 9, g > 0 peaks at
 * w = -w_i: light keeps travelling the way it went (forward scattering). */
static double hg_phase(double g, double w_dot_wi)
{
    return (1.0 - g * g) / (4.0 * M_PI * pow(1.0 + g * g + 2.0 * g * w_dot_wi, 1.5));
}

/* In-scattered radiance for an anisotropic phase function (Eq. 5 third term
 * with Eq. 9, g != 0). The scattered radiance depends on the direction of
 * interest, which for a pinhole view v at a point p is fixed by p itself:
 * the light travels from p to the camera centre o_v, w = (o_v - p)/|o_v - p|.
 * So each view sees its own grid over the same nodes:
 *   S_vc(p) = sum_d W_d L_c(p <- u_d) / sum_d W_d,  W_d = p(w, u_d),
 * with L_c(p <- u_d) the same emission-absorption march as orc_inscatter
 * (light arriving from u_d) and the phase weights normalised over the
 * directions, so that a radiance field equal in every direction scatters
 * into itself (the discrete phase function integrates to one). At g = 0
 * this is orc_inscatter for every view. A node at a camera centre has no
 * direction of interest and takes the mean (g = 0).
 * S [V][C][M^3]. */
int orc_inscatter_phase(const orc_grid *g, const orc_camera *cams, int32_t V, int32_t C, const double *em,
                        const double *sig, int32_t s_res, int32_t n_dirs, double s_step, double phase_g,
                        double *S)
{
    if (s_res < 2 || n_dirs < 1 || n_dirs > 256 || C > 16 || !(fabs(phase_g) < 1.0)) return -1;
    long N = grid_nodes(g);
    orc_grid sg;
    for (int a = 0; a < 3; ++a) { sg.n[a] = s_res; sg.lo[a] = g->lo[a]; sg.hi[a] = g->hi[a]; }
    double hs[3];
    grid_spacing(&sg, hs);
    double ds = s_step * grid_min_spacing(&sg);
    long M3 = (long)s_res * s_res * s_res;
    /* camera centres o = -R^T t */
    double *centre = (double *)malloc(sizeof(double) * 3 * V);
    if (!centre) return -2;
    for (int v = 0; v < V; ++v)
        for (int a = 0; a < 3; ++a)
            centre[3 * v + a] = -(cams[v].R[0 * 3 + a] * cams[v].t[0] + cams[v].R[1 * 3 + a] * cams[v].t[1] +
                                  cams[v].R[2 * 3 + a] * cams[v].t[2]);
#pragma omp parallel for schedule(static)
    for (long m = 0; m < M3; ++m) {
        int mx = (int)(m % s_res), my = (int)((m / s_res) % s_res), mz = (int)(m / ((long)s_res * s_res));
        double p[3];
        scat_node(g, hs, mx, my, mz, p);
        double L[256][16];
        double U[256][3];
        for (int dd = 0; dd < n_dirs; ++dd) {
            double tn, tf;
            fib_dir(dd, n_dirs, U[dd]);
            for (int ch = 0; ch < C; ++ch) L[dd][ch] = 0.0;
            if (!ray_box(g->lo, g->hi, p, U[dd], &tn, &tf)) continue;
            int K = n_segments(tn, tf, ds);
            double T = 1.0;
            for (int k = 0; k < K; ++k) {
                double t, len, x[3], q[3];
                segment(tn, tf, ds, k, &t, &len);
                for (int a = 0; a < 3; ++a) x[a] = p[a] + t * U[dd][a];
                to_grid_coords(g, x, q);
                double s = trilerp(g, sig, q);
                if (s < 0.0) s = 0.0;
                double wgt = T * len * phi(s * len);
                for (int ch = 0; ch < C; ++ch) L[dd][ch] += wgt * trilerp(g, em + (long)ch * N, q);
                T *= exp(-s * len);
            }
        }
        for (int v = 0; v < V; ++v) {
            double w[3], nrm = 0.0;
            for (int a = 0; a < 3; ++a) {
                w[a] = centre[3 * v + a] - p[a];
                nrm += w[a] * w[a];
            }
            nrm = sqrt(nrm);
            double num[16], den = 0.0;
            for (int ch = 0; ch < C; ++ch) num[ch] = 0.0;
            for (int dd = 0; dd < n_dirs; ++dd) {
                double W = 1.0;
                if (nrm > 0.0)
                    W = hg_phase(phase_g, (w[0] * U[dd][0] + w[1] * U[dd][1] + w[2] * U[dd][2]) / nrm);
                den += W;
                for (int ch = 0; ch < C; ++ch) num[ch] += W * L[dd][ch];
            }
            for (int ch = 0; ch < C; ++ch) S[((long)v * C + ch) * M3 + m] = num[ch] / den;
        }
    }
    free(centre);
    return 0;
}

/* ------------------------------------------------------ back-projection */

static double *alloc_private(int nt, long n)
{
    return (double *)calloc((size_t)nt * (size_t)n, sizeof(double));
}

static void reduce_private(const double *priv, int nt, long n, double *out)
{
    for (long i = 0; i < n; ++i) out[i] = 0.0;
    for (int t = 0; t < nt; ++t)
        for (long i = 0; i < n; ++i) out[i] += priv[(long)t * n + i];
}

/* Transpose of the linear emission -> image map A of orc_render (extinction
 * fixed, no in-scattering, no background):
 *   delta_c[j] = sum_rays sum_k res_c(ray) * T_k Delta_k phi_k * w_j(x_k),
 * w_j = trilinear weight of key point j at sample x_k. Written as a scatter
 * over rays and samples into per-thread private accumulators (Alg. 2 adds
 * the adjustment of the eight key points of every sample). res
 * [V][C][H][W], delta [C][N]. */
int orc_backproject_adjoint(const orc_grid *g, const orc_camera *cams, int32_t V, int32_t C,
                            double step_vox, const double *sig, const double *res, double *delta)
{
    double ds = step_vox * grid_min_spacing(g);
    long N = grid_nodes(g);
    int nt = n_threads();
    double *priv = alloc_private(nt, (long)C * N);
    if (!priv) return -2;
    for (int v = 0; v < V; ++v) {
        const orc_camera *c = &cams[v];
        long HW = (long)c->width * c->height;
#pragma omp parallel num_threads(nt)
        {
            double *acc = priv + (long)thread_id() * C * N;
#pragma omp for schedule(static)
            for (long p = 0; p < HW; ++p) {
                int u = (int)(p % c->width), vv = (int)(p / c->width);
                double o[3], d[3], tn, tf;
                camera_ray(c, u, vv, o, d);
                if (!ray_box(g->lo, g->hi, o, d, &tn, &tf)) continue;
                int K = n_segments(tn, tf, ds);
                double T = 1.0;
                for (int k = 0; k < K; ++k) {
                    double t, len, x[3], q[3], w[8];
                    long idx[8];
                    segment(tn, tf, ds, k, &t, &len);
                    for (int a = 0; a < 3; ++a) x[a] = o[a] + t * d[a];
                    to_grid_coords(g, x, q);
                    double s = trilerp(g, sig, q);
                    if (s < 0.0) s = 0.0;
                    double gw = T * len * phi(s * len);
                    stencil(g, q, idx, w, NULL, NULL);
                    for (int ch = 0; ch < C; ++ch) {
                        double y = res[((long)v * C + ch) * HW + p];
                        for (int cr = 0; cr < 8; ++cr) acc[(long)ch * N + idx[cr]] += y * gw * w[cr];
                    }
                    T *= exp(-s * len);
                }
            }
        }
    }
    reduce_private(priv, nt, (long)C * N, delta);
    free(priv);
    return 0;
}

/* Paper's adjustment (Eq. 10-12 with G(s) = 1): every sample s of every ray
 * adds to each of its eight neighbouring key points j
 *   A_js = alpha_l * dL(x, y) * (1 - tau)^k * exp(-alpha_d * D(j, s)),
 * with dL the colour residual of the ray's pixel (source minus rendered),
 * k the 0-based order of the sample counted from the ray's entry into the
 * volume (Eq. 12 with its exponent k - 1 for 1-based order) and D the
 * Euclidean distance in voxel units. dL [V][C][H][W], delta [C][N]. */
int orc_backproject_paper(const orc_grid *g, const orc_camera *cams, int32_t V, int32_t C,
                          double step_vox, double alpha_l, double alpha_d, double tau,
                          const double *dL, double *delta)
{
    double ds = step_vox * grid_min_spacing(g);
    long N = grid_nodes(g);
    int nt = n_threads();
    double *priv = alloc_private(nt, (long)C * N);
    if (!priv) return -2;
    for (int v = 0; v < V; ++v) {
        const orc_camera *c = &cams[v];
        long HW = (long)c->width * c->height;
#pragma omp parallel num_threads(nt)
        {
            double *acc = priv + (long)thread_id() * C * N;
#pragma omp for schedule(static)
            for (long p = 0; p < HW; ++p) {
                int u = (int)(p % c->width), vv = (int)(p / c->width);
                double o[3], d[3], tn, tf;
                camera_ray(c, u, vv, o, d);
                if (!ray_box(g->lo, g->hi, o, d, &tn, &tf)) continue;
                int K = n_segments(tn, tf, ds);
                for (int k = 0; k < K; ++k) {
                    double t, len, x[3], q[3], w[8], f[3];
                    long idx[8];
                    int cell[3];
                    segment(tn, tf, ds, k, &t, &len);
                    for (int a = 0; a < 3; ++a) x[a] = o[a] + t * d[a];
                    to_grid_coords(g, x, q);
                    stencil(g, q, idx, w, f, cell);
                    double tr = pow(1.0 - tau, (double)k);
                    for (int cr = 0; cr < 8; ++cr) {
                        double ddx = f[0] - (double)(cr & 1);
                        double ddy = f[1] - (double)((cr >> 1) & 1);
                        double ddz = f[2] - (double)((cr >> 2) & 1);
                        double D = sqrt(ddx * ddx + ddy * ddy + ddz * ddz);
                        double a = alpha_l * tr * exp(-alpha_d * D);
                        for (int ch = 0; ch < C; ++ch)
                            acc[(long)ch * N + idx[cr]] += a * dL[((long)v * C + ch) * HW + p];
                    }
                }
            }
        }
    }
    reduce_private(priv, nt, (long)C * N, delta);
    free(priv);
    return 0;
}

/* ------------------------------------------------------- differentiation */

/* dphi/dx for phi(x) = (1 - e^{-x}) / x: (e^{-x}(1 + x) - 1) / x^2, by its
 * Taylor series -1/2 + x/3 - x^2/8 + x^3/30 - x^4/144 near 0. */
static double dphi(double x)
{
    if (fabs(x) < 1e-3) return -0.5 + x / 3.0 - x * x / 8.0 + x * x * x / 30.0 - x * x * x * x / 144.0;
    return (exp(-x) * (1.0 + x) - 1.0) / (x * x);
}

/* Gradient of a scalar loss L through orc_render, given dL/dI (dLdI
 * [V][C][H][W]): d_em [C][N] = dL/d emission, d_sig [N] = dL/d extinction at
 * the key points. The in-scattered radiance S is held fixed (its dependence
 * on the volume is not differentiated).
 * Per ray and channel, with a_k = sigma_k Delta_k and the render of
 * orc_render,
 *   dI_c/d eps_kc   = T_k Delta_k phi(a_k)
 *   dI_c/d sigma_k  = T_k (albedo S_kc Delta_k phi(a_k) + j_kc Delta_k^2 phi'(a_k))
 *                     - Delta_k (sum_{k' > k} T_k' c_k'c + T_K L_bg)
 * (sigma_k enters its own segment and attenuates everything behind it), and
 * sample derivatives reach key point j through the trilinear weight w_j(x_k).
 * sigma_k = max(0, trilinear sigma) passes the derivative where the
 * trilinear value is >= 0. Plain per-ray arrays, private accumulators per
 * thread reduced in thread order. */
int orc_render_grad(const orc_grid *g, const orc_camera *cams, int32_t V, int32_t C, double step_vox,
                    double albedo, double background, const double *em, const double *sig,
                    int32_t s_res, const double *S, int32_t s_views, const double *dLdI, double *d_em,
                    double *d_sig)
{
    double ds = step_vox * grid_min_spacing(g);
    long N = grid_nodes(g);
    orc_grid sg;
    if (S)
        for (int a = 0; a < 3; ++a) { sg.n[a] = s_res; sg.lo[a] = g->lo[a]; sg.hi[a] = g->hi[a]; }
    int nt = n_threads();
    double *priv = alloc_private(nt, (long)(C + 1) * N);
    if (!priv) return -2;
    int rc = 0;
    for (int v = 0; v < V; ++v) {
        const orc_camera *c = &cams[v];
        long HW = (long)c->width * c->height;
        const double *Sv = S ? view_grid(S, s_views, v, C, s_res) : NULL;
#pragma omp parallel num_threads(nt)
        {
            double *acc = priv + (long)thread_id() * (C + 1) * N;
#pragma omp for schedule(static)
            for (long p = 0; p < HW; ++p) {
                int u = (int)(p % c->width), vv = (int)(p / c->width);
                double o[3], d[3], tn, tf;
                camera_ray(c, u, vv, o, d);
                if (!ray_box(g->lo, g->hi, o, d, &tn, &tf)) continue;
                int K = n_segments(tn, tf, ds);
                /* forward pass: keep every sample's state */
                double *T = (double *)malloc(sizeof(double) * (K + 1));
                double *len = (double *)malloc(sizeof(double) * K);
                double *sg_k = (double *)malloc(sizeof(double) * K);
                double *pos = (double *)malloc(sizeof(double) * K);     /* 1 if trilinear sigma >= 0 */
                double *j = (double *)malloc(sizeof(double) * K * C);
                double *Sk = (double *)malloc(sizeof(double) * K * C);
                double *q = (double *)malloc(sizeof(double) * K * 3);
                if (!T || !len || !sg_k || !pos || !j || !Sk || !q) {
                    free(T); free(len); free(sg_k); free(pos); free(j); free(Sk); free(q);
                    rc = -2;
                    continue;
                }
                T[0] = 1.0;
                for (int k = 0; k < K; ++k) {
                    double t, x[3];
                    segment(tn, tf, ds, k, &t, &len[k]);
                    for (int a = 0; a < 3; ++a) x[a] = o[a] + t * d[a];
                    to_grid_coords(g, x, &q[3 * k]);
                    double sraw = trilerp(g, sig, &q[3 * k]);
                    pos[k] = sraw >= 0.0 ? 1.0 : 0.0;
                    sg_k[k] = sraw > 0.0 ? sraw : 0.0;
                    for (int ch = 0; ch < C; ++ch) {
                        Sk[k * C + ch] = 0.0;
                        if (S && albedo != 0.0) {
                            double qs[3];
                            to_grid_coords(&sg, x, qs);
                            Sk[k * C + ch] = trilerp(&sg, Sv + (long)ch * s_res * s_res * s_res, qs);
                        }
                        j[k * C + ch] = trilerp(g, em + (long)ch * N, &q[3 * k]) + albedo * sg_k[k] * Sk[k * C + ch];
                    }
                    T[k + 1] = T[k] * exp(-sg_k[k] * len[k]);
                }
                /* backward pass: suffix radiance behind each sample */
                double R[16];
                for (int ch = 0; ch < C; ++ch) R[ch] = T[K] * background;
                for (int k = K - 1; k >= 0; --k) {
                    double a = sg_k[k] * len[k];
                    double ph = phi(a), dph = dphi(a);
                    long idx[8];
                    double w[8];
                    stencil(g, &q[3 * k], idx, w, NULL, NULL);
                    double dsig = 0.0;
                    for (int ch = 0; ch < C; ++ch) {
                        double y = dLdI[((long)v * C + ch) * HW + p];
                        double de = T[k] * len[k] * ph;
                        double dsg = T[k] * (albedo * Sk[k * C + ch] * len[k] * ph + j[k * C + ch] * len[k] * len[k] * dph)
                                     - len[k] * R[ch];
                        dsig += y * dsg;
                        for (int cr = 0; cr < 8; ++cr) acc[(long)ch * N + idx[cr]] += y * de * w[cr];
                        R[ch] += T[k] * j[k * C + ch] * len[k] * ph;
                    }
                    dsig *= pos[k];
                    for (int cr = 0; cr < 8; ++cr) acc[(long)C * N + idx[cr]] += dsig * w[cr];
                }
                free(T); free(len); free(sg_k); free(pos); free(j); free(Sk); free(q);
            }
        }
    }
    double *tmp = (double *)malloc(sizeof(double) * (C + 1) * N);
    if (!tmp) { free(priv); return -2; }
    reduce_private(priv, nt, (long)(C + 1) * N, tmp);
    memcpy(d_em, tmp, sizeof(double) * C * N);
    memcpy(d_sig, tmp + (long)C * N, sizeof(double) * N);
    free(tmp);
    free(priv);
    return rc;
}

/* ------------------------------------------------------ reconstruction */

static long images_size(const orc_camera *cams, int V, int C)
{
    return (long)V * C * cams[0].width * cams[0].height;
}

/* Iterative reconstruction of the emission (Sec. 3 overview: start from the
 * given volume, render, compare with the frames, adjust, repeat; Alg. 2).
 * R = A 1 (row sums) and Cs = A^T 1 (column sums) of the linear emission ->
 * image map A at the fixed extinction; rows and columns with zero sum are
 * skipped. I(e) is the full render including in-scattering, whose grid S (one
 * per view when phase_g != 0, orc_inscatter_phase) is
 * recomputed from the current volume at the start of every iteration and
 * held fixed within it.
 *
 * mode 0, SART (simultaneous over all views, i.e. SIRT):
 *   e <- e + lambda * Cs^{-1} A^T R^{-1} (F - I(e)), optionally clamped at 0.
 * mode 1, the paper's adjustment (Eq. 10-11, G = 1):
 *   e <- e + delta_paper(F - I(e)), optionally clamped at 0.
 * mode 2, multiplicative EM update (ML-EM, Shepp and Vardi 1982):
 *   e <- e * (1 + lambda * (A^T q / Cs - 1)),  q = F / I(e) on rays with
 *   I > 0 and q = 1 elsewhere.
 * frames [V][C][H][W], sig [N], em_io [C][N].
 * resid_out (optional, [iters]) receives sum (F - I)^2 before each update. */
int orc_reconstruct(const orc_grid *g, const orc_camera *cams, int32_t V, int32_t C,
                    double step_vox, double albedo, double background, int32_t s_res,
                    int32_t n_dirs, double s_step, double phase_g, const double *frames, const double *sig,
                    double *em_io, int32_t iters, int32_t mode, double lambda,
                    int32_t clamp_nonneg, double alpha_l, double alpha_d, double tau,
                    double *resid_out)
{
    long N = grid_nodes(g);
    long NI = images_size(cams, V, C);
    long HW = (long)cams[0].width * cams[0].height;
    for (int v = 1; v < V; ++v)
        if (cams[v].width != cams[0].width || cams[v].height != cams[0].height) return -1;
    double *img = (double *)malloc(sizeof(double) * NI);
    double *y = (double *)malloc(sizeof(double) * NI);
    double *delta = (double *)malloc(sizeof(double) * C * N);
    double *rows = (double *)malloc(sizeof(double) * V * HW);
    double *cols = (double *)malloc(sizeof(double) * N);
    double *ones_n = (double *)malloc(sizeof(double) * N);
    double *ones_img = (double *)malloc(sizeof(double) * V * HW);
    long M3 = (long)s_res * s_res * s_res;
    long n_grids = phase_g != 0.0 ? V : 1;
    double *S = (albedo != 0.0 && s_res >= 2) ? (double *)malloc(sizeof(double) * n_grids * C * M3) : NULL;
    int rc = 0;
    if (!img || !y || !delta || !rows || !cols || !ones_n || !ones_img ||
        (albedo != 0.0 && s_res >= 2 && !S)) { rc = -2; goto done; }

    if (mode == 0 || mode == 2) {
        /* R = A 1 and Cs = A^T 1 for the fixed extinction. */
        for (long i = 0; i < N; ++i) ones_n[i] = 1.0;
        for (long i = 0; i < V * HW; ++i) ones_img[i] = 1.0;
        rc = orc_render(g, cams, V, 1, step_vox, 0.0, 0.0, ones_n, sig, 0, NULL, 0, rows, NULL);
        if (rc) goto done;
        rc = orc_backproject_adjoint(g, cams, V, 1, step_vox, sig, ones_img, cols);
        if (rc) goto done;
    }
    for (int it = 0; it < iters; ++it) {
        if (S) {
            rc = phase_g != 0.0
                     ? orc_inscatter_phase(g, cams, V, C, em_io, sig, s_res, n_dirs, s_step, phase_g, S)
                     : orc_inscatter(g, C, em_io, sig, s_res, n_dirs, s_step, S);
            if (rc) goto done;
        }
        rc = orc_render(g, cams, V, C, step_vox, albedo, background, em_io, sig, s_res, S, phase_g != 0.0, img, NULL);
        if (rc) goto done;
        double r2 = 0.0;
        for (long i = 0; i < NI; ++i) {
            double r = frames[i] - img[i];
            r2 += r * r;
        }
        if (resid_out) resid_out[it] = r2;
        if (mode == 0 || mode == 2) {
            for (int v = 0; v < V; ++v)
                for (int ch = 0; ch < C; ++ch)
                    for (long p = 0; p < HW; ++p) {
                        long i = ((long)v * C + ch) * HW + p;
                        double R = rows[(long)v * HW + p];
                        if (mode == 0)
                            y[i] = R > 0.0 ? (frames[i] - img[i]) / R : 0.0;
                        else
                            y[i] = img[i] > 0.0 ? frames[i] / img[i] : 1.0;
                    }
            rc = orc_backproject_adjoint(g, cams, V, C, step_vox, sig, y, delta);
            if (rc) goto done;
            for (int ch = 0; ch < C; ++ch)
                for (long j = 0; j < N; ++j) {
                    if (!(cols[j] > 0.0)) continue;
                    double e = em_io[(long)ch * N + j];
                    if (mode == 0)
                        e += lambda * delta[(long)ch * N + j] / cols[j];
                    else
                        e *= 1.0 + lambda * (delta[(long)ch * N + j] / cols[j] - 1.0);
                    if (clamp_nonneg && e < 0.0) e = 0.0;
                    em_io[(long)ch * N + j] = e;
                }
        } else {
            for (long i = 0; i < NI; ++i) y[i] = frames[i] - img[i];
            rc = orc_backproject_paper(g, cams, V, C, step_vox, alpha_l, alpha_d, tau, y, delta);
            if (rc) goto done;
            for (long i = 0; i < (long)C * N; ++i) {
                double e = em_io[i] + delta[i];
                if (clamp_nonneg && e < 0.0) e = 0.0;
                em_io[i] = e;
            }
        }
    }
done:
    free(img); free(y); free(delta); free(rows); free(cols); free(ones_n); free(ones_img); free(S);
    return rc;
}

/* ------------------------------------------------- paper variants (f3) */

/* Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
 * easy as 1, 2, 3", SC 2011): ten rounds of two 32x32 -> 64-bit multiplies
 * with the key bumped by the Weyl constants between rounds. */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c[1] ^ k0, n1 = lo1, n2 = hi0 ^ c[3] ^ k1, n3 = lo0;
        c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    for (int i = 0; i < 4; ++i) out[i] = c[i];
}

/* G(s) of Eq. 11 for sample k of pixel `pix` of view v at iteration `it`:
 * 1 + g_sigma * z, z standard normal by Box-Muller from the first two
 * Philox words, u = (word + 1/2) / 2^32. */
double orc_sample_gain(uint64_t seed, int32_t it, int32_t v, int64_t pix, int32_t k, double g_sigma)
{
    if (g_sigma == 0.0) return 1.0;
    uint32_t ctr[4] = {(uint32_t)k, (uint32_t)pix, (uint32_t)v, (uint32_t)it};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t o[4];
    orc_philox4x32_10(ctr, key, o);
    double u1 = ((double)o[0] + 0.5) / 4294967296.0, u2 = ((double)o[1] + 0.5) / 4294967296.0;
    double z = sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
    return 1.0 + g_sigma * z;
}

/* Flame pixels (Sec. 4.1): a pixel is a flame pixel when any channel of the
 * frame exceeds the threshold. frames [V][C][H][W], mask [V][H][W] (1 or 0). */
void orc_flame_mask(const double *frames, int32_t V, int32_t C, long HW, double threshold, double *mask)
{
    for (int v = 0; v < V; ++v)
        for (long p = 0; p < HW; ++p) {
            double m = 0.0;
            for (int c = 0; c < C; ++c)
                if (frames[((long)v * C + c) * HW + p] > threshold) m = 1.0;
            mask[(long)v * HW + p] = m;
        }
}

/* Visual hull (Alg. 1): every flame ray of view v tags the key points around
 * it -- the eight corners of every cell holding one of its samples -- with
 * bit v; a key point is inside when it carries the bits of all views.
 * mask [V][H][W], inside [N] (1 or 0). */
int orc_visual_hull(const orc_grid *g, const orc_camera *cams, int32_t V, double step_vox, const double *mask,
                    int32_t *inside)
{
    if (V > 64) return -1;
    double ds = step_vox * grid_min_spacing(g);
    long N = grid_nodes(g);
    uint64_t *tag = (uint64_t *)calloc((size_t)N, sizeof(uint64_t));
    if (!tag) return -2;
    for (int v = 0; v < V; ++v) {
        const orc_camera *c = &cams[v];
        long HW = (long)c->width * c->height;
        for (long p = 0; p < HW; ++p) {
            if (mask[(long)v * HW + p] == 0.0) continue;
            int u = (int)(p % c->width), vv = (int)(p / c->width);
            double o[3], d[3], tn, tf;
            camera_ray(c, u, vv, o, d);
            if (!ray_box(g->lo, g->hi, o, d, &tn, &tf)) continue;
            int K = n_segments(tn, tf, ds);
            for (int k = 0; k < K; ++k) {
                double t, len, x[3], q[3], w[8];
                long idx[8];
                segment(tn, tf, ds, k, &t, &len);
                for (int a = 0; a < 3; ++a) x[a] = o[a] + t * d[a];
                to_grid_coords(g, x, q);
                stencil(g, q, idx, w, NULL, NULL);
                for (int cr = 0; cr < 8; ++cr) tag[idx[cr]] |= (uint64_t)1 << v;
            }
        }
    }
    uint64_t all = V == 64 ? ~(uint64_t)0 : (((uint64_t)1 << V) - 1);
    for (long j = 0; j < N; ++j) inside[j] = tag[j] == all;
    free(tag);
    return 0;
}

typedef struct {
    int32_t mode;            /* 0 SART, 1 paper (Eq. 10-11), 2 EM */
    double lambda;
    int32_t clamp_nonneg;
    double alpha_l, alpha_d, tau;
    double g_sigma;          /* std of the gain G(s) of Eq. 11 (paper mode); 0: G = 1 */
    uint64_t seed;
    int32_t use_mask;        /* adjust with flame rays only */
    double flame_threshold;
    int32_t use_hull;        /* reconstruct key points inside the visual hull only */
    double outside_value;    /* value given to key points outside the hull */
    double stop_tol;         /* > 0: stop when successive image errors differ by less */
    int32_t subsets;         /* > 1: ordered subsets of views (view v in subset v mod subsets) */
} orc_recon_params;

/* Paper-mode adjustment with per-sample gains and a ray mask (Eq. 10-12):
 * the same as orc_backproject_paper with A_js multiplied by G(s) and rays
 * with mask 0 skipped. */
static int backproject_paper_ext(const orc_grid *g, const orc_camera *cams, int32_t V, int32_t C,
                                 double step_vox, const orc_recon_params *rp, int32_t it,
                                 const double *mask, const double *dL, double *delta)
{
    double ds = step_vox * grid_min_spacing(g);
    long N = grid_nodes(g);
    int nt = n_threads();
    double *priv = alloc_private(nt, (long)C * N);
    if (!priv) return -2;
    for (int v = 0; v < V; ++v) {
        const orc_camera *c = &cams[v];
        long HW = (long)c->width * c->height;
#pragma omp parallel num_threads(nt)
        {
            double *acc = priv + (long)thread_id() * C * N;
#pragma omp for schedule(static)
            for (long p = 0; p < HW; ++p) {
                if (mask && mask[(long)v * HW + p] == 0.0) continue;
                int u = (int)(p % c->width), vv = (int)(p / c->width);
                double o[3], d[3], tn, tf;
                camera_ray(c, u, vv, o, d);
                if (!ray_box(g->lo, g->hi, o, d, &tn, &tf)) continue;
                int K = n_segments(tn, tf, ds);
                for (int k = 0; k < K; ++k) {
                    double t, len, x[3], q[3], w[8], f[3];
                    long idx[8];
                    segment(tn, tf, ds, k, &t, &len);
                    for (int a = 0; a < 3; ++a) x[a] = o[a] + t * d[a];
                    to_grid_coords(g, x, q);
                    stencil(g, q, idx, w, f, NULL);
                    double gain = orc_sample_gain(rp->seed, it, v, p, k, rp->g_sigma);
                    double tr = pow(1.0 - rp->tau, (double)k);
                    for (int cr = 0; cr < 8; ++cr) {
                        double ddx = f[0] - (double)(cr & 1);
                        double ddy = f[1] - (double)((cr >> 1) & 1);
                        double ddz = f[2] - (double)((cr >> 2) & 1);
                        double D = sqrt(ddx * ddx + ddy * ddy + ddz * ddz);
                        double a = gain * rp->alpha_l * tr * exp(-rp->alpha_d * D);
                        for (int ch = 0; ch < C; ++ch)
                            acc[(long)ch * N + idx[cr]] += a * dL[((long)v * C + ch) * HW + p];
                    }
                }
            }
        }
    }
    reduce_private(priv, nt, (long)C * N, delta);
    free(priv);
    return 0;
}

/* Reconstruction with the paper's variants on top of orc_reconstruct:
 *  - flame mask (Sec. 4.1): only flame rays enter the adjustment (their rows
 *    of A for SART / EM, including the column sums);
 *  - visual hull (Alg. 1): key points outside keep outside_value and are never
 *    adjusted;
 *  - gain G(s) of Eq. 11 in paper mode;
 *  - stop rule (Sec. 3): E_it = RMS of F - I over the adjusted pixels before
 *    the update of iteration it; stop before updating when it >= 1 and
 *    |E_{it-1} - E_it| < stop_tol.
 * iters_done receives the number of updates made; resid_out[it] = E_it. */
/* Ordered subsets (the classic per-view form of SART, OS-EM): the views are
 * split into n subsets (view v in subset v mod n) and every iteration
 * updates the volume once per subset in order, each update being the
 * simultaneous step of the chosen rule restricted to that subset's rays:
 * its own row sums and its own column sums C_j^s = (A_s^T 1)_j. The
 * in-scatter grid is recomputed at the start of each iteration and held
 * fixed over its subsets. Flame mask and visual hull apply as in
 * orc_reconstruct_ext; the gains G(s) and the stop rule are not combined
 * with subsets. */
static int reconstruct_subsets(const orc_grid *g, const orc_camera *cams, int32_t V, int32_t C, double step_vox,
                               double albedo, double background, int32_t s_res, int32_t n_dirs, double s_step,
                               double phase_g, const double *frames, const double *sig, double *em_io,
                               int32_t iters, const orc_recon_params *rp, int32_t *iters_done)
{
    const int ns = rp->subsets;
    if (ns > V || rp->stop_tol > 0.0 || rp->g_sigma != 0.0) return -1;
    long N = grid_nodes(g);
    long HW = (long)cams[0].width * cams[0].height;
    long M3 = (long)s_res * s_res * s_res;
    int vmax = (V + ns - 1) / ns;
    orc_camera *sc = (orc_camera *)malloc(sizeof(orc_camera) * vmax);
    double *F = (double *)malloc(sizeof(double) * vmax * C * HW);
    double *img = (double *)malloc(sizeof(double) * vmax * C * HW);
    double *y = (double *)malloc(sizeof(double) * vmax * C * HW);
    double *rows = (double *)malloc(sizeof(double) * vmax * HW);
    double *mask_all = (double *)malloc(sizeof(double) * V * HW);
    double *mask = (double *)malloc(sizeof(double) * vmax * HW);
    double *cols = (double *)malloc(sizeof(double) * ns * N);
    double *ones_n = (double *)malloc(sizeof(double) * N);
    double *delta = (double *)malloc(sizeof(double) * C * N);
    int32_t *inside = (int32_t *)malloc(sizeof(int32_t) * N);
    long n_grids = phase_g != 0.0 ? V : 1;
    double *S = (albedo != 0.0 && s_res >= 2) ? (double *)malloc(sizeof(double) * n_grids * C * M3) : NULL;
    double *Ss = (albedo != 0.0 && s_res >= 2 && phase_g != 0.0) ? (double *)malloc(sizeof(double) * vmax * C * M3)
                                                                  : NULL;
    int rc = 0, done = 0;
    if (!sc || !F || !img || !y || !rows || !mask_all || !mask || !cols || !ones_n || !delta || !inside ||
        (albedo != 0.0 && s_res >= 2 && !S) || (albedo != 0.0 && s_res >= 2 && phase_g != 0.0 && !Ss)) {
        rc = -2;
        goto done;
    }
    if (rp->use_mask) orc_flame_mask(frames, V, C, HW, rp->flame_threshold, mask_all);
    else for (long i = 0; i < V * HW; ++i) mask_all[i] = 1.0;
    if (rp->use_hull) {
        rc = orc_visual_hull(g, cams, V, step_vox, mask_all, inside);
        if (rc) goto done;
        for (int ch = 0; ch < C; ++ch)
            for (long j = 0; j < N; ++j)
                if (!inside[j]) em_io[(long)ch * N + j] = rp->outside_value;
    } else {
        for (long j = 0; j < N; ++j) inside[j] = 1;
    }
    for (long i = 0; i < N; ++i) ones_n[i] = 1.0;
    /* gather subset s: its cameras, frames and mask rows; returns its view count */
#define TAKE_SUBSET(s_)                                                                            \
    int vs = 0;                                                                                    \
    for (int v = (s_); v < V; v += ns, ++vs) {                                                     \
        sc[vs] = cams[v];                                                                          \
        memcpy(F + (long)vs * C * HW, frames + (long)v * C * HW, sizeof(double) * C * HW);         \
        memcpy(mask + (long)vs * HW, mask_all + (long)v * HW, sizeof(double) * HW);                \
    }
    if (rp->mode == 0 || rp->mode == 2)
        for (int s = 0; s < ns; ++s) {
            TAKE_SUBSET(s)
            rc = orc_backproject_adjoint(g, sc, vs, 1, step_vox, sig, mask, cols + (long)s * N);
            if (rc) goto done;
        }
    for (int it = 0; it < iters; ++it) {
        if (S) {
            rc = phase_g != 0.0
                     ? orc_inscatter_phase(g, cams, V, C, em_io, sig, s_res, n_dirs, s_step, phase_g, S)
                     : orc_inscatter(g, C, em_io, sig, s_res, n_dirs, s_step, S);
            if (rc) goto done;
        }
        for (int s = 0; s < ns; ++s) {
            TAKE_SUBSET(s)
            const double *Sv = S;
            if (S && phase_g != 0.0) {
                for (int k = 0, v = s; v < V; v += ns, ++k)
                    memcpy(Ss + (long)k * C * M3, S + (long)v * C * M3, sizeof(double) * C * M3);
                Sv = Ss;
            }
            rc = orc_render(g, sc, vs, C, step_vox, albedo, background, em_io, sig, s_res, Sv, phase_g != 0.0,
                            img, NULL);
            if (rc) goto done;
            if (rp->mode == 0 || rp->mode == 2) {
                rc = orc_render(g, sc, vs, 1, step_vox, 0.0, 0.0, ones_n, sig, 0, NULL, 0, rows, NULL);
                if (rc) goto done;
            }
            for (int v = 0; v < vs; ++v)
                for (int ch = 0; ch < C; ++ch)
                    for (long p = 0; p < HW; ++p) {
                        long i = ((long)v * C + ch) * HW + p;
                        double m = mask[(long)v * HW + p];
                        if (rp->mode == 0) {
                            double R = rows[(long)v * HW + p];
                            y[i] = (m != 0.0 && R > 0.0) ? (F[i] - img[i]) / R : 0.0;
                        } else if (rp->mode == 2) {
                            y[i] = m != 0.0 ? (img[i] > 0.0 ? F[i] / img[i] : 1.0) : 0.0;
                        } else {
                            y[i] = m != 0.0 ? F[i] - img[i] : 0.0;
                        }
                    }
            if (rp->mode == 1)
                rc = orc_backproject_paper(g, sc, vs, C, step_vox, rp->alpha_l, rp->alpha_d, rp->tau, y, delta);
            else
                rc = orc_backproject_adjoint(g, sc, vs, C, step_vox, sig, y, delta);
            if (rc) goto done;
            const double *cs = cols + (long)s * N;
            for (int ch = 0; ch < C; ++ch)
                for (long j = 0; j < N; ++j) {
                    if (!inside[j]) continue;
                    double e = em_io[(long)ch * N + j];
                    if (rp->mode == 1) {
                        e += delta[(long)ch * N + j];
                    } else {
                        if (!(cs[j] > 0.0)) continue;
                        if (rp->mode == 0) e += rp->lambda * delta[(long)ch * N + j] / cs[j];
                        else e *= 1.0 + rp->lambda * (delta[(long)ch * N + j] / cs[j] - 1.0);
                    }
                    if (rp->clamp_nonneg && e < 0.0) e = 0.0;
                    em_io[(long)ch * N + j] = e;
                }
        }
        ++done;
    }
#undef TAKE_SUBSET
done:
    if (iters_done) *iters_done = done;
    free(sc); free(F); free(img); free(y); free(rows); free(mask_all); free(mask); free(cols); free(ones_n);
    free(delta); free(inside); free(S); free(Ss);
    return rc;
}

int orc_reconstruct_ext(const orc_grid *g, const orc_camera *cams, int32_t V, int32_t C, double step_vox,
                        double albedo, double background, int32_t s_res, int32_t n_dirs, double s_step,
                        double phase_g, const double *frames, const double *sig, double *em_io, int32_t iters,
                        const orc_recon_params *rp, double *resid_out, int32_t *iters_done)
{
    if (rp->subsets > 1)
        return reconstruct_subsets(g, cams, V, C, step_vox, albedo, background, s_res, n_dirs, s_step, phase_g,
                                   frames, sig, em_io, iters, rp, iters_done);
    long N = grid_nodes(g);
    long HW = (long)cams[0].width * cams[0].height;
    long NI = (long)V * C * HW;
    double *img = (double *)malloc(sizeof(double) * NI);
    double *y = (double *)malloc(sizeof(double) * NI);
    double *delta = (double *)malloc(sizeof(double) * C * N);
    double *rows = (double *)malloc(sizeof(double) * V * HW);
    double *cols = (double *)malloc(sizeof(double) * N);
    double *ones_n = (double *)malloc(sizeof(double) * N);
    double *mask = (double *)malloc(sizeof(double) * V * HW);
    int32_t *inside = (int32_t *)malloc(sizeof(int32_t) * N);
    long M3 = (long)s_res * s_res * s_res;
    long n_grids = phase_g != 0.0 ? V : 1;
    double *S = (albedo != 0.0 && s_res >= 2) ? (double *)malloc(sizeof(double) * n_grids * C * M3) : NULL;
    int rc = 0, done = 0;
    double prev_err = 0.0;
    if (!img || !y || !delta || !rows || !cols || !ones_n || !mask || !inside ||
        (albedo != 0.0 && s_res >= 2 && !S)) { rc = -2; goto done; }
    if (rp->use_mask) orc_flame_mask(frames, V, C, HW, rp->flame_threshold, mask);
    else for (long i = 0; i < V * HW; ++i) mask[i] = 1.0;
    if (rp->use_hull) {
        rc = orc_visual_hull(g, cams, V, step_vox, mask, inside);
        if (rc) goto done;
        for (int ch = 0; ch < C; ++ch)
            for (long j = 0; j < N; ++j)
                if (!inside[j]) em_io[(long)ch * N + j] = rp->outside_value;
    } else {
        for (long j = 0; j < N; ++j) inside[j] = 1;
    }
    if (rp->mode == 0 || rp->mode == 2) {
        for (long i = 0; i < N; ++i) ones_n[i] = 1.0;
        rc = orc_render(g, cams, V, 1, step_vox, 0.0, 0.0, ones_n, sig, 0, NULL, 0, rows, NULL);
        if (rc) goto done;
        rc = orc_backproject_adjoint(g, cams, V, 1, step_vox, sig, mask, cols);
        if (rc) goto done;
    }
    for (int it = 0; it < iters; ++it) {
        if (S) {
            rc = phase_g != 0.0
                     ? orc_inscatter_phase(g, cams, V, C, em_io, sig, s_res, n_dirs, s_step, phase_g, S)
                     : orc_inscatter(g, C, em_io, sig, s_res, n_dirs, s_step, S);
            if (rc) goto done;
        }
        rc = orc_render(g, cams, V, C, step_vox, albedo, background, em_io, sig, s_res, S, phase_g != 0.0, img, NULL);
        if (rc) goto done;
        double r2 = 0.0, cnt = 0.0;
        for (int v = 0; v < V; ++v)
            for (int ch = 0; ch < C; ++ch)
                for (long p = 0; p < HW; ++p) {
                    if (mask[(long)v * HW + p] == 0.0) continue;
                    long i = ((long)v * C + ch) * HW + p;
                    r2 += (frames[i] - img[i]) * (frames[i] - img[i]);
                    cnt += 1.0;
                }
        double err = cnt > 0.0 ? sqrt(r2 / cnt) : 0.0;
        if (resid_out) resid_out[it] = err;
        if (rp->stop_tol > 0.0 && it >= 1 && fabs(prev_err - err) < rp->stop_tol) break;
        prev_err = err;
        for (int v = 0; v < V; ++v)
            for (int ch = 0; ch < C; ++ch)
                for (long p = 0; p < HW; ++p) {
                    long i = ((long)v * C + ch) * HW + p;
                    double m = mask[(long)v * HW + p];
                    double R = rows[(long)v * HW + p];
                    if (rp->mode == 0) y[i] = (m != 0.0 && R > 0.0) ? (frames[i] - img[i]) / R : 0.0;
                    else if (rp->mode == 2) y[i] = (m != 0.0) ? (img[i] > 0.0 ? frames[i] / img[i] : 1.0) : 0.0;
                    else y[i] = m != 0.0 ? frames[i] - img[i] : 0.0;
                }
        if (rp->mode == 1)
            rc = backproject_paper_ext(g, cams, V, C, step_vox, rp, it, mask, y, delta);
        else
            rc = orc_backproject_adjoint(g, cams, V, C, step_vox, sig, y, delta);
        if (rc) goto done;
        for (int ch = 0; ch < C; ++ch)
            for (long j = 0; j < N; ++j) {
                if (!inside[j]) continue;
                double e = em_io[(long)ch * N + j];
                if (rp->mode == 1) {
                    e += delta[(long)ch * N + j];
                } else {
                    if (!(cols[j] > 0.0)) continue;
                    if (rp->mode == 0) e += rp->lambda * delta[(long)ch * N + j] / cols[j];
                    else e *= 1.0 + rp->lambda * (delta[(long)ch * N + j] / cols[j] - 1.0);
                }
                if (rp->clamp_nonneg && e < 0.0) e = 0.0;
                em_io[(long)ch * N + j] = e;
            }
        ++done;
    }
done:
    if (iters_done) *iters_done = done;
    free(img); free(y); free(delta); free(rows); free(cols); free(ones_n); free(mask); free(inside); free(S);
    return rc;
}

/* --------------------------------------------------------- temperature */

/* Planck's law (Eq. 13): spectral radiance of a black body at wavelength
 * lambda [m] and temperature T [K], with exact SI constants and the vacuum
 * speed of light (the flame's refractive index is taken as 1). */
double orc_planck(double lambda, double T)
{
    const double h = 6.62607015e-34, c = 2.99792458e8, kb = 1.380649e-23;
    double x = h * c / (lambda * kb * T);
    return 2.0 * h * c * c / pow(lambda, 5.0) / expm1(x);
}

/* Band radiance: integral of B(lambda, T) * exp(-(lambda - mu)^2 / (2 s^2))
 * over [mu - 6 s, mu + 6 s] by composite Simpson with `panels` panels
 * (rounded up to even). mu, s in nm; the result is per metre of
 * wavelength times nm. */
double orc_band_radiance(double T, double mu_nm, double std_nm, int32_t panels)
{
    if (panels < 2) panels = 2;
    if (panels & 1) ++panels;
    double a = mu_nm - 6.0 * std_nm, b = mu_nm + 6.0 * std_nm;
    double hstep = (b - a) / panels, s = 0.0;
    for (int i = 0; i <= panels; ++i) {
        double l = a + i * hstep;
        double z = (l - mu_nm) / std_nm;
        double f = orc_planck(l * 1e-9, T) * exp(-0.5 * z * z);
        double wgt = (i == 0 || i == panels) ? 1.0 : ((i & 1) ? 4.0 : 2.0);
        s += wgt * f;
    }
    return s * hstep / 3.0;
}

/* Colour-temperature mapping (Sec. 3.3 "Temperature Reconstruction"):
 * B_c(T) = band_c(T) / band_ch(t_norm), tabulated at lut_size temperatures
 * evenly spaced over [t_min, t_max]. lut [3][lut_size]. */
int orc_temp_lut(const orc_temp_params *tp, double *lut)
{
    int L = tp->lut_size;
    if (L < 2) return -1;
    double norm = orc_band_radiance(tp->t_norm, tp->band_nm[tp->channel], tp->band_std_nm, tp->panels);
    for (int c = 0; c < 3; ++c)
        for (int i = 0; i < L; ++i) {
            double T = tp->t_min + (tp->t_max - tp->t_min) * (double)i / (double)(L - 1);
            lut[(long)c * L + i] = orc_band_radiance(T, tp->band_nm[c], tp->band_std_nm, tp->panels) / norm;
        }
    return 0;
}

/* LUT lookup with linear interpolation; T clamped to the LUT domain. */
static double lut_lookup(const orc_temp_params *tp, const double *row, double T)
{
    int L = tp->lut_size;
    double pos = (T - tp->t_min) / (tp->t_max - tp->t_min) * (double)(L - 1);
    if (pos < 0.0) pos = 0.0;
    if (pos > (double)(L - 1)) pos = (double)(L - 1);
    int i = (int)floor(pos);
    if (i > L - 2) i = L - 2;
    double f = pos - (double)i;
    return row[i] * (1.0 - f) + row[i + 1] * f;
}

/* Per key point: emission eps_c = B_c(T) from the LUT (em may be NULL) and
 * extinction sigma = sigma_max * max(0, (T - soot_t0) / soot_span) (soot
 * load grows with temperature). em [3][n], sig [n]. */
void orc_temp_map(const orc_temp_params *tp, const double *lut, const double *T, long n, double *em,
                  double *sig)
{
    int L = tp->lut_size;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) {
        if (em)
            for (int c = 0; c < 3; ++c) em[(long)c * n + i] = lut_lookup(tp, lut + (long)c * L, T[i]);
        if (sig) {
            double s = (T[i] - tp->soot_t0) / tp->soot_span;
            sig[i] = tp->sigma_max * (s > 0.0 ? s : 0.0);
        }
    }
}

/* Inverse of the fit channel's LUT: e clamped to [B(t_min), B(t_max)], the
 * bracketing entries found by bisection (the table is increasing), then
 * linear interpolation between their temperatures. */
void orc_temp_invert(const orc_temp_params *tp, const double *lut, const double *e, long n, double *T)
{
    int L = tp->lut_size;
    const double *row = lut + (long)tp->channel * L;
    double dT = (tp->t_max - tp->t_min) / (double)(L - 1);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) {
        double x = e[i];
        if (x <= row[0]) { T[i] = tp->t_min; continue; }
        if (x >= row[L - 1]) { T[i] = tp->t_max; continue; }
        int lo = 0, hi = L - 1; /* row[lo] <= x < row[hi] */
        while (hi - lo > 1) {
            int mid = (lo + hi) / 2;
            if (row[mid] <= x) lo = mid; else hi = mid;
        }
        double f = (x - row[lo]) / (row[hi] - row[lo]);
        T[i] = tp->t_min + ((double)lo + f) * dT;
    }
}

/* Temperature reconstruction (Sec. 3.3: reconstruct the green channel as in
 * the colour reconstruction, then read the temperature off the
 * colour-temperature mapping). The extinction follows the temperature
 * (soot load), so it is re-derived from the current estimate every
 * iteration. Per iteration:
 *   1. eps = B_ch(T), sigma = sigma(T)                  (map)
 *   2. I = A(sigma) eps                                 (render, fit channel)
 *   3. q = F_ch / I on rays with I > 0, else 1          (residual ratio)
 *   4. N = A(sigma)^T q, Cs = A(sigma)^T 1              (back-projection)
 *   5. eps <- clamp(eps * (1 + lambda (N / Cs - 1)), B_ch(t_min), B_ch(t_max))
 *   6. T = B_ch^{-1}(eps)                               (inverse map)
 * The multiplicative (EM) step keeps each voxel's relative change bounded.
 * An additive step (eps += N'/Cs with residual differences) is unstable
 * here: near t_min the map T(eps) is so steep that round-off in eps moves
 * T, hence sigma, by amounts whose effect on the frames grows without bound
 * from one iteration to the next.
 * frames [V][3][H][W] (only the fit channel is read), T_io [N]. */
int orc_temperature_fit(const orc_grid *g, const orc_camera *cams, int32_t V, double step_vox,
                        const orc_temp_params *tp, const double *lut, const double *frames,
                        double *T_io, int32_t iters, double lambda, double *resid_out)
{
    long N = grid_nodes(g);
    long HW = (long)cams[0].width * cams[0].height;
    int L = tp->lut_size;
    const double *row = lut + (long)tp->channel * L;
    double *eps = (double *)malloc(sizeof(double) * N);
    double *sig = (double *)malloc(sizeof(double) * N);
    double *cols = (double *)malloc(sizeof(double) * N);
    double *num = (double *)malloc(sizeof(double) * N);
    double *img = (double *)malloc(sizeof(double) * V * HW);
    double *q = (double *)malloc(sizeof(double) * V * HW);
    double *ones_img = (double *)malloc(sizeof(double) * V * HW);
    double *tmp = (double *)malloc(sizeof(double) * 3 * N);
    int rc = 0;
    if (!eps || !sig || !cols || !num || !img || !q || !ones_img || !tmp) {
        rc = -2;
        goto done;
    }
    for (long i = 0; i < V * HW; ++i) ones_img[i] = 1.0;
    for (int it = 0; it < iters; ++it) {
        orc_temp_map(tp, lut, T_io, N, tmp, sig);
        memcpy(eps, tmp + (long)tp->channel * N, sizeof(double) * N);
        rc = orc_render(g, cams, V, 1, step_vox, 0.0, 0.0, eps, sig, 0, NULL, 0, img, NULL);
        if (rc) goto done;
        double r2 = 0.0;
        for (int v = 0; v < V; ++v)
            for (long p = 0; p < HW; ++p) {
                double F = frames[((long)v * 3 + tp->channel) * HW + p];
                double I = img[(long)v * HW + p];
                r2 += (F - I) * (F - I);
                q[(long)v * HW + p] = I > 0.0 ? F / I : 1.0;
            }
        if (resid_out) resid_out[it] = r2;
        rc = orc_backproject_adjoint(g, cams, V, 1, step_vox, sig, q, num);
        if (rc) goto done;
        rc = orc_backproject_adjoint(g, cams, V, 1, step_vox, sig, ones_img, cols);
        if (rc) goto done;
        for (long j = 0; j < N; ++j) {
            double e = eps[j];
            if (cols[j] > 0.0) e *= 1.0 + lambda * (num[j] / cols[j] - 1.0);
            if (e < row[0]) e = row[0];
            if (e > row[L - 1]) e = row[L - 1];
            eps[j] = e;
        }
        orc_temp_invert(tp, lut, eps, N, T_io);
    }
done:
    free(eps); free(sig); free(cols); free(num); free(img); free(q); free(ones_img); free(tmp);
    return rc;
}

/* ------------------------------------------ volume dimensions (Sec. 4.2) */

/* Volume dimensions from the cameras (Sec. 4.2): project the eight vertices
 * of the box [lo, hi] into every image; each of the twelve box edges spans
 * |du| and |dv| pixels; n_max[a] = the largest of these spans over the four
 * edges along axis a and over all views, and the volume gets
 * ceil(n_max[a] / alpha) voxels along a (alpha = 1.5 in the paper), i.e.
 * one key point more. An edge with an end point on or behind a camera's
 * image plane (z_c <= 0) is skipped for that camera. Returns -1 when no
 * edge along some axis projects into any view. voxels [3] (x, y, z),
 * n_max [3] (optional). */
int orc_suggest_grid(const orc_camera *cams, int32_t V, const double lo[3], const double hi[3], double alpha,
                     int32_t voxels[3], double *n_max)
{
    if (V < 1 || !(alpha > 0.0)) return -1;
    double best[3] = {0.0, 0.0, 0.0};
    for (int v = 0; v < V; ++v) {
        const orc_camera *c = &cams[v];
        double uv[8][2];
        int front[8];
        for (int corner = 0; corner < 8; ++corner) {
            double x[3] = {(corner & 1) ? hi[0] : lo[0], (corner & 2) ? hi[1] : lo[1], (corner & 4) ? hi[2] : lo[2]};
            double xc[3];
            for (int r = 0; r < 3; ++r)
                xc[r] = c->R[3 * r] * x[0] + c->R[3 * r + 1] * x[1] + c->R[3 * r + 2] * x[2] + c->t[r];
            front[corner] = xc[2] > 0.0;
            uv[corner][0] = front[corner] ? c->fx * (xc[0] / xc[2]) + c->cx : 0.0;
            uv[corner][1] = front[corner] ? c->fy * (xc[1] / xc[2]) + c->cy : 0.0;
        }
        /* the edge along axis a joins corners that differ only in bit a */
        for (int a = 0; a < 3; ++a)
            for (int corner = 0; corner < 8; ++corner) {
                if (corner & (1 << a)) continue;
                int other = corner | (1 << a);
                if (!front[corner] || !front[other]) continue;
                double du = fabs(uv[other][0] - uv[corner][0]), dv = fabs(uv[other][1] - uv[corner][1]);
                double span = du > dv ? du : dv;
                if (span > best[a]) best[a] = span;
            }
    }
    for (int a = 0; a < 3; ++a) {
        if (!(best[a] > 0.0)) return -1;
        double n = ceil(best[a] / alpha);
        voxels[a] = n < 1.0 ? 1 : (int32_t)n;
        if (n_max) n_max[a] = best[a];
    }
    return 0;
}

int orc_num_threads(void) { return n_threads(); }

/* Threads the parallel loops use from now on (1 .. 32); results depend on
 * the count only through the fixed-order reduction of private sums. */
void orc_set_num_threads(int32_t n)
{
#ifdef _OPENMP
    omp_set_num_threads(n < 1 ? 1 : (n > ORC_MAX_THREADS ? ORC_MAX_THREADS : n));
#else
    (void)n;
#endif
}
