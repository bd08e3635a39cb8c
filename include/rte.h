/*
 * rte.h -- C ABI of librte, an MI355X (gfx950) implementation of the
 * iterative loop of radiative-transport flame volume reconstruction
 * (Shen et al., "Radiative Transport Based Flame Volume Reconstruction from
 * Videos", arXiv:1809.06417): render every camera view of a voxel volume by
 * perspective ray marching (Eq. 5-8, Sec. 3.3), compare with the captured
 * frames, back-project the residuals into a volume update (Eq. 10-11,
 * Alg. 2), and the same loop for the black-body temperature fit (Eq. 13,
 * Sec. 3.3 "Temperature Reconstruction").
 *
 * Conventions
 *  - Every array argument is a DEVICE pointer to FP32 (or int32 where
 *    stated), C-contiguous, owned by the caller. The library never frees or
 *    retains caller memory beyond the call.
 *  - Volumes are [channel][z][y][x] (x fastest) on a node-centred grid: nx,
 *    ny, nz key points at the voxel vertices (Sec. 3.3 "Key points")
 *    spanning [bbox_min, bbox_max]; trilinear interpolation between them.
 *  - Cameras: x_cam = R x_world + t; pixel (u, v) has its centre at
 *    (u + 1/2, v + 1/2); u grows right, v down, the optical axis is +z_cam.
 *    All cameras of a plan share one width x height.
 *  - Images are [view][channel][v][u].
 *  - Calls are asynchronous on `stream` (a hipStream_t, NULL = default
 *    stream). Argument errors are detected before anything is enqueued.
 *    Execution errors surface at the caller's next synchronisation.
 *  - Return value: RTE_OK (0) or a negative RTE_ERR_* code; rte_last_error()
 *    gives a message. After an argument or budget error nothing was
 *    enqueued and in/out arrays are untouched.
 *  - A plan may be used by one stream at a time; distinct plans are
 *    independent. Hot calls never allocate device memory: every workspace
 *    is allocated by rte_plan_create.
 */
#ifndef RTE_H
#define RTE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RTE_OK 0
#define RTE_ERR_INVALID_ARG (-1)
#define RTE_ERR_BUDGET (-2)
#define RTE_ERR_HIP (-3)
#define RTE_ERR_UNSUPPORTED (-4)

/* Pinhole camera (perspective projection, Sec. 3.2; intrinsics and
 * extrinsics from calibration, Sec. 4.1). Double precision: the per-plan ray
 * table is derived from it in FP64. R is row-major. */
typedef struct {
    double fx, fy, cx, cy;
    double R[9];
    double t[3];
    int32_t width, height;
} rte_camera;

/* Node-centred grid of key points (Sec. 3.3): n >= 2 per axis. */
typedef struct {
    int32_t nx, ny, nz;
    double bbox_min[3], bbox_max[3];
} rte_grid;

/* Forward model (Eq. 5-9).
 *  channels      1 or 3 emission channels (R, G, B reconstructed together, Sec. 3).
 *  step_vox      sampling step along each ray in units of the smallest node
 *                spacing (Sec. 4.2 uses one voxel; 0.5 is the default here).
 *  albedo        sigma_s / sigma_t; 0 disables in-scattering.
 *  background    radiance behind the volume (0: dark capture, Sec. 4.1).
 *  scatter_res   nodes per axis of the in-scatter grid (>= 2 when albedo > 0).
 *  scatter_dirs  directions of the in-scatter quadrature (1..256).
 *  scatter_step  in-scatter march step in units of the in-scatter node spacing.
 *  flags         RTE_PLAN_* bits (RTE_PLAN_GRADIENTS: also allocate what
 *                rte_render_backward needs).
 *  phase_g       Henyey-Greenstein asymmetry g of Eq. 9, |g| < 1 (0: the
 *                isotropic phase function the paper uses). With g != 0 the
 *                in-scattered radiance depends on the direction towards the
 *                camera, so every view has its own in-scatter grid: the
 *                in-scatter arrays of rte_inscatter, rte_render and
 *                rte_render_forward/backward are [V][C][M][M][M] instead of
 *                [C][M][M][M]. */
typedef struct {
    int32_t channels;
    float step_vox;
    float albedo;
    float background;
    int32_t scatter_res;
    int32_t scatter_dirs;
    float scatter_step;
    int32_t flags;
    float phase_g;
} rte_render_params;

#define RTE_PLAN_GRADIENTS 1

/* Back-projection weights. */
typedef enum {
    RTE_BP_ADJOINT = 0, /* exact transpose of the linear emission -> image map */
    RTE_BP_PAPER = 1    /* adjustment values of Eq. 10 with the transparency of Eq. 12 */
} rte_bp_mode;

/* Volume update rule of the reconstruction loop. */
typedef enum {
    RTE_UPDATE_SART = 0,  /* e += lambda * (A^T 1)^-1 A^T (A 1)^-1 (F - I), all views at once */
    RTE_UPDATE_PAPER = 1, /* e += sum_s A_js (Eq. 10-11 with G = 1) */
    RTE_UPDATE_MLEM = 2   /* e *= 1 + lambda * (A^T (F / I) / A^T 1 - 1) */
} rte_update;

/* Reconstruction parameters.
 *  update        an rte_update value.
 *  lambda        relaxation (SART, MLEM); 1 is the plain step.
 *  clamp_nonneg  clamp the emission at 0 after each update.
 *  alpha_l, alpha_d, tau   paper-mode constants of Eq. 10 and Eq. 12
 *                (Sec. 5.1 uses 0.001, 1, 0.05; D is measured in voxels).
 *  g_sigma, seed paper mode: every sample's adjustment is weighted by a gain
 *                G(s) = 1 + g_sigma * z (Eq. 11), z standard normal from a
 *                Philox-4x32-10 counter keyed by seed, counter (k, pixel,
 *                view, iteration) and Box-Muller; g_sigma = 0 gives G = 1.
 *  use_mask, flame_threshold   only flame rays -- pixels where some channel
 *                of the frame exceeds the threshold (Sec. 4.1) -- enter the
 *                adjustment (and the column sums).
 *  use_hull, outside_value     reconstruct only key points inside the visual
 *                hull of the flame rays (Alg. 1); the others are set to
 *                outside_value and left alone (the paper uses a small
 *                negative number).
 *  stop_tol      > 0: stop once the image RMS over the adjusted pixels of two
 *                successive iterations differs by less (Sec. 3; the paper
 *                uses 0.01 on its 0-255 scale); iters is then a maximum.
 *  ordered_subsets  0 or 1: every update uses all views at once. n > 1
 *                (n <= views): ordered subsets, the classic per-view form
 *                of SART (n = views) and OS-EM: view v belongs to subset
 *                v mod n, and an iteration makes n updates in subset order,
 *                each the rule above restricted to the subset's rays (its
 *                own row and column sums). The in-scatter grid is refreshed
 *                once per iteration. Not combined with stop_tol or g_sigma
 *                (RTE_ERR_UNSUPPORTED) nor with jobs. */
typedef struct {
    int32_t update;
    float lambda;
    int32_t clamp_nonneg;
    float alpha_l, alpha_d, tau;
    float g_sigma;
    uint64_t seed;
    int32_t use_mask;
    float flame_threshold;
    int32_t use_hull;
    float outside_value;
    float stop_tol;
    int32_t ordered_subsets;
} rte_recon_params;

/* Colour-temperature mapping (Eq. 13; Sec. 3.3). The LUT holds, at lut_size
 * temperatures evenly spaced over [t_min, t_max], the band radiances
 *   B_c(T) = int B(lambda, T) w_c(lambda) dlambda / int B(lambda, t_norm) w_ch(lambda) dlambda,
 * w_c a Gaussian band of centre band_nm[c] and standard deviation
 * band_std_nm, over the window of +-6 standard deviations around the
 * centre, integrated by composite 4-point Gauss-Legendre quadrature on
 * panels / 4 sub-intervals (built on the host in FP64; every band's window
 * must lie at positive wavelengths, else RTE_ERR_INVALID_ARG). Extinction follows
 * the soot load: sigma = sigma_max * max(0, (T - soot_t0) / soot_span).
 * `channel` is the fitted channel (1 = green, Sec. 3.3). */
typedef struct {
    float t_min, t_max, t_norm;
    float band_nm[3];
    float band_std_nm;
    int32_t lut_size;
    float sigma_max, soot_t0, soot_span;
    int32_t channel;
    int32_t panels;
} rte_temp_params;

typedef struct rte_plan rte_plan;

/* Build a plan for one grid and camera rig (host structs). Computes the ray
 * table on the device (per pixel: entry point, chord length and segment
 * count; Alg. 2 casts one ray per pixel) and allocates every workspace.
 * Synchronises `stream` once. Fails with RTE_ERR_BUDGET, allocating
 * nothing that it keeps, if the workspace would exceed hbm_budget_bytes
 * (0 = no limit). *out receives the plan. */
int rte_plan_create(rte_plan **out, const rte_grid *grid, const rte_camera *cams, int32_t ncams,
                    const rte_render_params *params, size_t hbm_budget_bytes, void *stream);

/* Upper bound of the device bytes rte_plan_create would allocate for these
 * arguments (host-side estimate; no device work). Returns 0 on invalid
 * arguments. */
size_t rte_plan_workspace_bytes(const rte_grid *grid, const rte_camera *cams, int32_t ncams,
                                const rte_render_params *params);

/* Device bytes actually held by the plan. */
size_t rte_plan_device_bytes(const rte_plan *plan);

/* Release the plan (synchronises its last stream first). NULL is ignored. */
void rte_plan_destroy(rte_plan *plan);

/* Number of march samples of one pass over all rays (sum of the segment
 * counts) and number of rays that hit the volume. */
int rte_plan_counts(const rte_plan *plan, uint64_t *samples, uint64_t *hit_rays);

/* Volume dimensions from the camera rig (Sec. 4.2, volume dimensions): the
 * eight corners of the box [bbox_min, bbox_max] are projected into every
 * view; along each axis a, n_max[a] = the largest pixel span max(|du|, |dv|)
 * of the four box edges parallel to a over all views, and the volume gets
 * ceil(n_max[a] / alpha) voxels (alpha = 1.5 in the paper), i.e. one key
 * point more, written to grid (with the box). An edge with an end point on
 * or behind a camera's image plane (camera z <= 0) does not count for that
 * camera. With the paper's sampling step of one voxel edge, pass
 * step_vox = 1 to rte_plan_create. Host only: no device work.
 * cams [ncams] (image sizes are not used), grid (written), n_max [3]
 * (written, may be NULL). Errors: RTE_ERR_INVALID_ARG for null pointers,
 * ncams < 1, alpha <= 0, an empty box, or an axis none of whose edges
 * projects into any view; grid is untouched then. */
int rte_suggest_grid(const rte_camera *cams, int32_t ncams, const double bbox_min[3],
                     const double bbox_max[3], double alpha, rte_grid *grid, double *n_max);

/* Export the ray table: t_near, t_far (world units along the unit ray
 * direction) and segment count K per pixel, [view][v][u] device arrays.
 * Rays that miss get K = 0 and t_near = t_far = 0. */
int rte_ray_table(rte_plan *plan, float *t_near, float *t_far, int32_t *nseg, void *stream);

/* Render every view (Eq. 5-8 along each ray, front to back):
 *   I_c = sum_k T_k j_kc Delta_k phi(sigma_k Delta_k) + T_K * background,
 *   T_{k+1} = T_k exp(-sigma_k Delta_k),  phi(x) = (1 - e^-x) / x,
 *   j_kc = eps_c(x_k) + albedo * sigma(x_k) * S_c(x_k),
 * with segment midpoints x_k, the last segment clipped at the exit.
 * emission [C][nz][ny][nx], extinction [nz][ny][nx] (>= 0),
 * inscatter [C][M][M][M] (M = scatter_res) or NULL (no in-scattering),
 * images [V][C][H][W] (written). */
int rte_render(rte_plan *plan, const float *emission, const float *extinction,
               const float *inscatter, float *images, void *stream);

/* rte_render without a plan, for callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc. It gives the images rte_render gives on a plan created from the
 * same grid, cameras and params (the same kernels, bitwise the same result),
 * and allocates nothing: the camera copy, ray table, tile list, packed
 * volume and packed in-scatter grid live in one device array of
 * RTE_STATIC_SCRATCH_BYTES that the library holds on every GPU it runs on
 * until the process ends. The first call on a device looks up the array's
 * address there (make it outside graph capture); every call then only
 * enqueues kernels on `stream` (the cameras travel in kernel arguments).
 * Limits: at most RTE_STATIC_MAX_VIEWS cameras (RTE_ERR_UNSUPPORTED), and the
 * workspaces, each rounded up to 256 bytes, must fit the array
 * (RTE_ERR_BUDGET): 136 V + 36 V W H + 4 V ceil(W/8) ceil(H/8)
 * + (16 for 3 channels, 8 for 1) nx ny nz + 16 M^3 (times V when
 * phase_g != 0; 0 without in-scattering) bytes -- e.g. a 128^3 RGB volume
 * seen by 8 views of 512x512 with a 32^3 in-scatter grid takes 110 MB.
 * Nothing is enqueued after an error. All calls on one GPU share the array
 * and each call overwrites it: calls that may overlap on one GPU (other
 * streams, other host threads) race, and the caller must order them.
 * Arguments: grid, cams, ncams and params as for rte_plan_create
 * (params->flags is ignored); emission, extinction, inscatter and images as
 * for rte_render. */
#define RTE_STATIC_SCRATCH_BYTES (128u << 20)
#define RTE_STATIC_MAX_VIEWS 16
int rte_render_static(const rte_grid *grid, const rte_camera *cams, int32_t ncams,
                      const rte_render_params *params, const float *emission, const float *extinction,
                      const float *inscatter, float *images, void *stream);

/* rte_render that also writes each ray's optical depth at its exit,
 * exit_optical_depth [V][H][W] (FP64, tau_K = sum_k sigma_k Delta_k over the
 * ray's samples, 0 for rays that miss the box; the exit transmittance is
 * exp(-tau_K)). rte_render_backward re-marches each ray backwards from it.
 * It is kept in FP64 rather than as the FP32 transmittance because
 * exp(-tau_K) leaves the FP32 range (underflows) beyond tau_K of about 87,
 * where the transmittance in front of the ray's first samples still
 * matters. */
int rte_render_forward(rte_plan *plan, const float *emission, const float *extinction,
                       const float *inscatter, float *images, double *exit_optical_depth,
                       void *stream);

/* Gradient of a scalar loss through the render of Eq. 5-8, given dL/dI.
 * For every ray a reverse march recovers the transmittance in front of each
 * sample from exit_optical_depth (tau_k = tau_{k+1} - sigma_k Delta_k in
 * FP64, T_k = exp(-tau_k); no per-sample state is kept from the forward
 * pass) and forms
 *   dI_c/d eps_k   = T_k Delta_k phi_k,
 *   dI_c/d sigma_k = T_k (albedo S_c Delta_k phi_k + j_c Delta_k^2 phi'_k)
 *                    - Delta_k (radiance behind sample k);
 * these reach the key points through the trilinear weights in an
 * atomics-free voxel-owned gather. The in-scatter grid is held fixed.
 * Needs a plan created with RTE_PLAN_GRADIENTS. emission [C][nz][ny][nx],
 * extinction [nz][ny][nx], inscatter as in rte_render, exit_optical_depth
 * from rte_render_forward on the same inputs, grad_images [V][C][H][W];
 * writes grad_emission [C][nz][ny][nx] and grad_extinction [nz][ny][nx]. */
int rte_render_backward(rte_plan *plan, const float *emission, const float *extinction,
                        const float *inscatter, const double *exit_optical_depth,
                        const float *grad_images, float *grad_emission, float *grad_extinction,
                        void *stream);

/* In-scattered radiance grid (Eq. 5 third term with the phase function of
 * Eq. 9): at each node p of an M^3 grid over the box, L_d(p) = the
 * emission-absorption march from p along each of scatter_dirs
 * spherical-Fibonacci directions u_d to the box exit (single scattering);
 * phase_g = 0: S(p) = mean_d L_d(p);
 * phase_g != 0: for each view v, S_v(p) = sum_d W_d L_d(p) / sum_d W_d with
 * W_d = p(w, u_d) of Eq. 9 and w the unit direction from p to camera v's
 * centre (a node at a camera centre takes W_d = 1).
 * emission [C][nz][ny][nx], extinction [nz][ny][nx], inscatter [C][M][M][M]
 * or [V][C][M][M][M] when phase_g != 0 (written). */
int rte_inscatter(rte_plan *plan, const float *emission, const float *extinction, float *inscatter,
                  void *stream);

/* Back-project per-pixel values into a per-key-point volume (Alg. 2
 * adjustment pass, computed as an atomics-free voxel-owned gather).
 *  RTE_BP_ADJOINT: delta = A^T residual, A the linear emission -> image map
 *    of rte_render at this extinction without in-scattering or background.
 *  RTE_BP_PAPER: delta_j = sum over samples s touching j of
 *    alpha_l * residual * (1 - tau)^k * exp(-alpha_d * D(j, s))   (Eq. 10, 12;
 *    k = 0-based sample order from the ray's entry, D in voxels); `params`
 *    supplies alpha_l, alpha_d, tau and may be NULL for ADJOINT.
 * extinction [nz][ny][nx] (ADJOINT only; may be NULL for PAPER),
 * residual [V][C][H][W], delta [C][nz][ny][nx] (written). */
int rte_backproject(rte_plan *plan, const float *extinction, const float *residual, float *delta,
                    int32_t mode, const rte_recon_params *params, void *stream);

/* Iterative colour reconstruction (Sec. 3: render, compare with the frames,
 * adjust the volume; repeated `iters` times). The extinction is known and
 * fixed; in-scattering (albedo > 0) is recomputed from the current emission
 * at the start of every iteration and held fixed within it. Row and column
 * sums of A are computed once per call.
 * frames [V][C][H][W], extinction [nz][ny][nx], emission [C][nz][ny][nx]
 * (in: start volume, out: result; warm start = pass the previous result). */
int rte_reconstruct(rte_plan *plan, const float *frames, const float *extinction, float *emission,
                    int32_t iters, const rte_recon_params *params, void *stream);

/* Jobs: the reconstruction loop of rte_reconstruct split so that several
 * plans can advance together, one iteration at a time (used by the serving
 * loop; continuous batching at iteration granularity).
 *
 * rte_job_begin opens a job on a plan: uploads the start volume -- or, with
 * emission == NULL, keeps the emission already resident in the plan from its
 * previous job (warm start) -- and the frame's extinction, and prepares the
 * flame mask and visual hull as rte_reconstruct does. frames
 * [V][C][H][W] stays owned by the caller and must stay valid until
 * rte_job_end. params->stop_tol must be 0 and params->ordered_subsets <= 1
 * (RTE_ERR_UNSUPPORTED otherwise).
 * rte_job_step advances every listed plan (1..64 distinct plans with open
 * jobs, one channel count, update rule and scattering setting) by one
 * iteration with one launch per phase covering all of them (with
 * in-scattering, one launch per march pass and reduce computes every plan's
 * grid; its arguments are staged in the first listed plan), except that the
 * first step of a SART or EM job runs on its own (its render also stores the
 * per-sample weights and its gather the column sums, as the first iteration
 * of rte_reconstruct does); each plan's result is bitwise the one it would
 * get alone and the one rte_reconstruct gives. The batched launch arguments
 * go through a staging buffer of the first batched plan (the first listed
 * plan past its first step, or any paper-rule plan): issue all steps that
 * share it on one stream. With timing on, the three batched launches are
 * charged to that plan (RTE_KERNEL_RENDER, _GATHER, _UPDATE), a first step's
 * launches to its own plan, the batched in-scatter to the first listed plan
 * (RTE_KERNEL_INSCATTER).
 * Errors: RTE_ERR_INVALID_ARG for a plan without an open job or listed twice,
 * RTE_ERR_UNSUPPORTED for more than 64 plans or mixed settings; no plan is
 * advanced then.
 * rte_job_end copies the result to emission [C][nz][ny][nx] (may be NULL;
 * the volume also stays resident in the plan) and closes the job. */
int rte_job_begin(rte_plan *plan, const float *frames, const float *extinction, const float *emission,
                  const rte_recon_params *params, void *stream);
int rte_job_step(rte_plan *const *plans, int32_t n, void *stream);
int rte_job_end(rte_plan *plan, float *emission, void *stream);

/* Updates made by the last rte_reconstruct on this plan and, when its stop
 * rule was on, the image RMS of each rendered iteration: n_errors receives
 * how many were recorded, at most max_errors are copied to errors (either
 * may be NULL). */
int rte_reconstruct_stats(const rte_plan *plan, int32_t *iters_done, int32_t *n_errors, float *errors,
                          int32_t max_errors);

/* Flame-pixel mask (Sec. 4.1): mask [V][H][W] = 1 where some channel of
 * frames [V][C][H][W] exceeds threshold, else 0 (C = the plan's channels). */
int rte_flame_mask(rte_plan *plan, const float *frames, float threshold, float *mask, void *stream);

/* Visual hull (Alg. 1): inside [nz][ny][nx] (int32) = 1 for key points that,
 * for every view, are a corner of a cell holding a sample of a flame ray;
 * flame rays are the pixels where mask [V][H][W] is non-zero (NULL: every
 * pixel). At most 64 views. */
int rte_visual_hull(rte_plan *plan, const float *mask, int32_t *inside, void *stream);

/* Temperature fit (Sec. 3.3): per iteration, map T -> (eps_ch, sigma) through
 * the LUT, render the fitted channel, back-project the frame/render ratio
 * (multiplicative EM step; params->update is ignored), clamp eps_ch to the
 * LUT range and invert the LUT to get T. The plan must have channels = 1.
 * frames [V][3][H][W] (only temp->channel is read), temperature
 * [nz][ny][nx] in Kelvin (in: start, out: result). */
int rte_reconstruct_temperature(rte_plan *plan, const float *frames, float *temperature,
                                int32_t iters, const rte_recon_params *params,
                                const rte_temp_params *temp, void *stream);

/* Colour-temperature map alone: emission [3][nz][ny][nx] = B_c(T) (may be
 * NULL) and extinction [nz][ny][nx] = sigma(T) (may be NULL) from
 * temperature [nz][ny][nx]. */
int rte_temperature_map(rte_plan *plan, const float *temperature, float *emission,
                        float *extinction, const rte_temp_params *temp, void *stream);

/* Inverse of the fitted channel's map: temperature = B_ch^-1(clamp(e)) by
 * bisection of the LUT and linear interpolation; e [nz][ny][nx]. */
int rte_temperature_invert(rte_plan *plan, const float *e, float *temperature,
                           const rte_temp_params *temp, void *stream);

/* Copy of the FP32 LUT the device uses, [3][lut_size] host array (for
 * inspection); lut_size must equal temp->lut_size. Synchronous. */
int rte_temperature_lut(rte_plan *plan, const rte_temp_params *temp, float *lut_host,
                        int32_t lut_size);

/* Per-kernel timing: when enabled, every launch of the plan is bracketed by
 * HIP events on the launch stream. rte_plan_kernel_time synchronises on the
 * recorded events and returns the total milliseconds and launch count of
 * kernel `kernel` (RTE_KERNEL_* below) since the last reset. */
enum {
    RTE_KERNEL_RAYS = 0,
    RTE_KERNEL_RENDER = 1,
    RTE_KERNEL_INSCATTER = 2,
    RTE_KERNEL_GATHER = 3,
    RTE_KERNEL_UPDATE = 4,
    RTE_KERNEL_TEMP_MAP = 5,
    RTE_KERNEL_PACK = 6,
    RTE_KERNEL_WEIGHTS = 7, /* render pass that only produces per-sample weights */
    RTE_KERNEL_COLSUM = 8,  /* reserved: the column sums A^T 1 come out of the first gather */
    RTE_KERNEL_ADJOINT = 9, /* reverse march of rte_render_backward */
    RTE_KERNEL_COUNT = 10
};
int rte_plan_set_timing(rte_plan *plan, int32_t enable);
int rte_plan_kernel_time(rte_plan *plan, int32_t kernel, double *total_ms, int64_t *launches);

/* Timing of some kernels only: bit k of `kernels` brackets the launches of
 * RTE_KERNEL k with events (each event adds a marker of a few microseconds to
 * the stream, so a measurement that needs one kernel's duration times only
 * that kernel); 0 turns timing off, and rte_plan_set_timing(plan, 1) equals
 * all bits set. Resets the totals like rte_plan_set_timing. Bits at or above
 * RTE_KERNEL_COUNT: RTE_ERR_INVALID_ARG. */
int rte_plan_set_timing_mask(rte_plan *plan, uint32_t kernels);

/* Message for the last non-zero return on this thread ("" if none). */
const char *rte_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* RTE_H */
