/*
 * gs.h - C ABI of the MI355X X-ray rasterizer and voxelizer of R^2-Gaussian
 * (radiative Gaussian splatting for tomographic reconstruction).
 *
 * A scene is a set of M "radiative Gaussians" G_i(x) = rho_i exp(-1/2 (x-p_i)^T
 * Sigma_i^{-1} (x-p_i)), Sigma_i = R_i S_i S_i^T R_i^T (paper Sec. 3.1, Eq. 3),
 * whose sum is the density field sigma(x) (Eq. 4).
 *
 *  - gs_project_*  render log-space X-ray projections, i.e. line integrals of
 *    sigma (Eq. 1), as a plain sum of rectified 2D Gaussians (Eq. 5-7, App. A
 *    Eq. 9-11), for cone-beam or parallel-beam views, and its gradient.
 *  - gs_voxelize_* evaluate sigma at voxel centres (Eq. 4, Sec. 3.2.2) and its
 *    gradient.
 *  - gs_loss_*     the training loss terms of Eq. 8: L1 + lambda D-SSIM on
 *    projections, 3D total variation on a voxel block, with gradients.
 *
 * Conventions for every entry point:
 *  - Array arguments are DEVICE pointers (FP32, C-contiguous, row-major) unless
 *    marked (host).  Structs passed by pointer are host memory, read during the
 *    call only.
 *  - All GPU work is enqueued on `stream`; results are ready when the stream
 *    reaches that point.  The projection and voxelization forward passes read
 *    back one integer (the number of tile entries) and so synchronize `stream`
 *    once, unless the plan is reserved (gs_plan_reserve); everything else is
 *    asynchronous.
 *  - Ownership: the caller owns every input, output and gradient buffer; the
 *    library never frees caller memory.  A plan owns only its workspace, which
 *    it obtains through the allocator given at creation (hipMalloc if NULL) and
 *    releases in gs_plan_destroy.  Distinct plans may be used from distinct
 *    threads; one plan must not be used by two calls at once.
 *  - Errors: every call returns a gs_status and never aborts.  Argument errors
 *    are detected on the host before any launch (GS_EINVAL).  After a non-OK
 *    status the outputs are undefined.  gs_last_error() gives a thread-local
 *    message for the last non-OK status.
 *  - Data problems are not errors: a Gaussian with a non-finite parameter, a
 *    scale <= 0 or a zero quaternion contributes nothing and gets a zero
 *    gradient; for cone beam a (view, Gaussian) pair whose centre lies within
 *    1e-3 L_SO of the source plane (or behind it) is culled the same way.
 *    Such Gaussians are counted by gs_plan_status.
 *  - cutoff: a (pixel, Gaussian) or (voxel, Gaussian) term is included iff its
 *    Mahalanobis distance q satisfies q <= cutoff^2 (inclusive).  cutoff must
 *    be > 0; INFINITY includes every term.  3 reproduces "3-sigma".
 */
#ifndef GS_H
#define GS_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__)
#define GS_API __attribute__((visibility("default")))
#else
#define GS_API
#endif

typedef enum {
  GS_OK = 0,
  GS_EINVAL = 1,        /* invalid argument (null pointer, bad size, bad geometry) */
  GS_ENOMEM = 2,        /* workspace allocation failed */
  GS_EOVERFLOW = 3,     /* more than 2^32-1 tile entries in one call (use fewer views per call),
                           or a reserved plan's call needed more entries than reserved */
  GS_EHIP = 4,          /* a HIP runtime call or kernel launch failed */
  GS_EUNSUPPORTED = 5   /* valid but unsupported request (e.g. detector wider than 16384) */
} gs_status;

typedef enum { GS_PARALLEL = 0, GS_CONE = 1 } gs_beam;

/* One view (host).  Scanner model of App. A: a world point x maps to scanner
 * coordinates t = W x + (0, 0, L_SO) (cone) or t = W x (parallel).  The rows of
 * W are the detector u axis (columns), the detector v axis (rows) and the
 * central ray direction; W must be a rotation.
 * Cone beam: the source is the scanner origin and the detector plane is at
 * depth L_SD; a centre projects to (L_SD t0/t2, L_SD t1/t2).  Parallel beam:
 * a centre projects to (t0, t1) (the limit L_SO -> infinity).
 * Pixel (column a, row b) samples the detector at its centre
 * ((a + 1/2 - width/2) pitch_u + off_u, (b + 1/2 - height/2) pitch_v + off_v).
 * Images are [height][width] per view. */
typedef struct {
  int32_t beam;            /* gs_beam */
  int32_t width, height;   /* detector pixels: columns, rows; 1..16384 */
  float pitch_u, pitch_v;  /* pixel size in world length units, > 0 */
  float off_u, off_v;      /* detector offset of the principal point */
  float rot[9];            /* W, row-major */
  float src_obj, src_det;  /* L_SO, L_SD (cone only): 0 < L_SO < L_SD */
} gs_view;

/* Voxel grid (host).  Voxel (i, j, k) centre: origin + ((i+1/2) sx, (j+1/2) sy,
 * (k+1/2) sz); volumes are [nz][ny][nx] (x fastest).  Sizes 1..16384. */
typedef struct {
  int32_t nx, ny, nz;
  float origin[3];
  float spacing[3];
} gs_grid;

/* Gaussian set (host struct of device pointers): mean [n][3], scale [n][3]
 * (post-activation standard deviations along the principal axes, > 0),
 * quat [n][4] as (w, x, y, z), Hamilton convention, normalised internally,
 * density [n] (central density rho, any real). */
typedef struct {
  int64_t n;
  const float *mean, *scale, *quat, *density;
} gs_gaussians;

/* Gradient outputs (host struct of device pointers, same shapes as
 * gs_gaussians).  Any pointer may be NULL to skip that output.  The quaternion
 * gradient is with respect to the unnormalised input quaternion. */
typedef struct {
  float *mean, *scale, *quat, *density;
} gs_grads;

typedef void *(*gs_alloc_fn)(size_t bytes, void *ctx);
typedef void (*gs_free_fn)(void *ptr, void *ctx);

/* Opaque workspace and saved forward state. */
typedef struct gs_plan gs_plan;

/* Create a plan.  alloc/free may both be NULL (then hipMalloc/hipFree on the
 * current device are used); otherwise both must be given and must return
 * device memory of the current device aligned to 256 bytes. */
GS_API gs_status gs_plan_create(gs_alloc_fn alloc, gs_free_fn free_fn, void *ctx, gs_plan **out);

/* Release the plan's workspace after synchronizing the last stream it used
 * (only that stream: other streams of the device are not waited for).  A
 * caller that used the plan on several streams orders them first. */
GS_API void gs_plan_destroy(gs_plan *plan);

/* Synchronize the plan's last stream and report the number of Gaussians (or
 * cone-beam (view, Gaussian) pairs) skipped by the last forward call, and the
 * number of tile entries the last projection and voxelization binnings of
 * the plan needed (summed; for a reserved plan the entries needed, also when
 * more than the reservation holds).  Either pointer may be NULL.  Returns
 * GS_EOVERFLOW (outputs filled) while a reserved plan records a call that
 * exceeded its reservation; gs_plan_check clears the record. */
GS_API gs_status gs_plan_status(gs_plan *plan, int64_t *skipped, int64_t *tile_entries);

/* Largest problem a reserved plan serves.  Zero counts skip that part. */
typedef struct {
  int64_t max_gaussians;     /* Gaussians per projection or voxelization call */
  int32_t max_views;         /* views per projection call (0: no projection part) */
  int32_t width, height;     /* detector size of those calls (calls may use smaller) */
  int64_t max_proj_entries;  /* (view, 16x16 tile, Gaussian) tile-list entries per call */
  int32_t nx, ny, nz;        /* largest voxel grid (0: no voxelization part) */
  int64_t max_vox_entries;   /* (8^3 tile, Gaussian) tile-list entries per call */
  int64_t max_tv_voxels;     /* voxels of the gs_loss_tv blocks (0: none) */
  int64_t max_records;       /* (view, Gaussian) pairs per projection call, summed over the
                                views (0: max_views x max_gaussians) */
  int32_t forward_only;      /* 1: no backward workspace; backward calls on the plan fail */
} gs_reserve;               /* gs_loss_image: stacks up to max_views x height x width */

/* Allocate the plan's whole workspace for problems up to r (synchronizes
 * `stream`) and switch the plan to reserved mode: from then on projection,
 * voxelization and loss calls on the plan never allocate and never
 * synchronize the stream (the binning no longer reads its entry count back),
 * so a caller can queue many calls ahead of the device or capture them in a
 * graph.  A call larger than the reservation fails with GS_EINVAL before any
 * launch.  If a call's tile lists exceed the reserved entries, the device
 * drops the excess entries and records the overflow: that call's image or
 * volume is incomplete and its backward writes no gradient (outputs
 * undefined).  The record is visible to the host without synchronizing: once
 * the device has set it, every projection or voxelization call on the plan
 * returns GS_EOVERFLOW before any launch, and so do gs_plan_status and
 * gs_plan_check (which synchronize), until gs_plan_check clears it.  Calls
 * queued before the device set it still run. */
GS_API gs_status gs_plan_reserve(gs_plan *plan, const gs_reserve *r, hipStream_t stream);

/* (host) Device bytes that gs_plan_reserve(r) allocates (its workspace, the
 * control words included), without allocating: for sizing reservations
 * against a memory budget. */
GS_API gs_status gs_plan_reserve_bytes(const gs_reserve *r, int64_t *bytes);

/* For a reserved plan: synchronize its last stream, report the largest
 * projection and voxel entry counts any call needed since the previous check
 * (either pointer may be NULL; filled also on GS_EOVERFLOW, so a caller can
 * reserve again from them) and return GS_EOVERFLOW if any call exceeded the
 * reservation since then.  Clears both records and the overflow state. */
GS_API gs_status gs_plan_check(gs_plan *plan, int64_t *max_proj_entries, int64_t *max_vox_entries);

/* (host) Fill a cone-beam view for gantry angle theta (radians) as in App. A,
 * Eq. 10: W rows (-sin t, cos t, 0), (0, 0, -1), (-cos t, -sin t, 0); square
 * pixels of size pitch, no offset.  The rotation is evaluated in double
 * precision and rounded to float. */
GS_API gs_status gs_view_cone(double theta, float src_obj, float src_det, int32_t width, int32_t height,
                       float pitch, gs_view *out);

/* Forward projection (Eq. 7 with App. A): image[v][b][a] =
 *   sum_i rho_hat_iv exp(-1/2 (x_ab - p_hat_iv)^T Sigma_hat_iv^{-1} (x_ab - p_hat_iv))
 * with rho_hat = sqrt(2 pi |Sigma_tilde| / |Sigma_hat|) rho (the rectified
 * density), over terms within the cutoff.  All views must share width and
 * height.  image: [n_views][height][width], overwritten.
 * plan: may be NULL (a temporary workspace is allocated and freed, and the
 * stream is synchronized); with a plan, the binning is kept for a following
 * gs_project_bwd on the same arguments.  Synchronizes `stream` once.
 * At most 2^28 - 1 Gaussians per projection call (GS_EUNSUPPORTED beyond). */
GS_API gs_status gs_project_fwd(const gs_gaussians *g, const gs_view *views, int32_t n_views,
                         float cutoff, float *image, gs_plan *plan, hipStream_t stream);

/* gs_project_fwd over several Gaussian sets in one launch: view v renders
 * models[view_model[v]] (host arrays: models [n_models], view_model
 * [n_views]), so requests for different resident models share the binning
 * and render launches.  Each view's image equals what gs_project_fwd gives
 * for that model and view up to the FP32 order of partial sums (a long tile
 * list may be split over workgroups differently).  The binning is not kept
 * for gs_project_bwd.  plan, stream and errors as for gs_project_fwd; at most
 * 2^28 - 1 Gaussians per model. */
GS_API gs_status gs_project_fwd_multi(const gs_gaussians *models, int32_t n_models,
                                      const int32_t *view_model, const gs_view *views,
                                      int32_t n_views, float cutoff, float *image, gs_plan *plan,
                                      hipStream_t stream);

/* Gradient of L = sum(grad_image * image) with respect to the Gaussian
 * parameters (the cutoff indicator is treated as locally constant).
 * grads are overwritten, or added to when accumulate != 0.
 * If plan holds the binning of a gs_project_fwd call with the same Gaussian
 * pointers, count, views and cutoff, it is reused (the Gaussian values must be
 * unchanged since then); otherwise the binning is recomputed (one stream
 * synchronization).  plan must not be NULL. */
GS_API gs_status gs_project_bwd(const gs_gaussians *g, const gs_view *views, int32_t n_views,
                         float cutoff, const float *grad_image, const gs_grads *grads,
                         int32_t accumulate, gs_plan *plan, hipStream_t stream);

/* Voxelization (Eq. 4): volume[k][j][i] = sum_i rho_i exp(-1/2 q_i(x_ijk))
 * over terms within the cutoff.  volume: [nz][ny][nx], overwritten.
 * plan may be NULL as for gs_project_fwd.  Synchronizes `stream` once. */
GS_API gs_status gs_voxelize_fwd(const gs_gaussians *g, const gs_grid *grid, float cutoff, float *volume,
                          gs_plan *plan, hipStream_t stream);

/* Gradient of L = sum(grad_volume * volume); same rules as gs_project_bwd. */
GS_API gs_status gs_voxelize_bwd(const gs_gaussians *g, const gs_grid *grid, float cutoff,
                          const float *grad_volume, const gs_grads *grads, int32_t accumulate,
                          gs_plan *plan, hipStream_t stream);

/* Projection loss of Eq. 8: L1 + lambda_ssim (1 - SSIM) between rendered and
 * measured stacks [n_img][h][w].  L1 is the mean absolute difference; SSIM is
 * the mean over all pixels and images of the SSIM map with an 11x11 Gaussian
 * window (sigma 1.5, normalised), zero padding, C1 = 0.01^2, C2 = 0.03^2.
 * loss_out (device, 3 floats): {total, l1, ssim}.
 * grad (device [n_img][h][w], may be NULL): d total / d render, overwritten.
 * The loss is the same number with or without grad (one kernel computes it).
 * Images of 2^29 pixels or more return GS_EUNSUPPORTED.
 * plan must not be NULL (holds the partial sums, one pair per wavefront of
 * the loss kernel, summed in a fixed order). */
GS_API gs_status gs_loss_image(const float *render, const float *measured, int32_t n_img, int32_t h,
                        int32_t w, float lambda_ssim, float *loss_out, float *grad, gs_plan *plan,
                        hipStream_t stream);

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Computes
 * exactly what gs_loss_image computes (same kernels, bitwise the same loss
 * and gradient), without a plan: the partial sums go to a static device
 * buffer inside the library, one per GPU, held until the process ends (2 MiB:
 * room for GS_LOSS_IMAGE_NOALLOC_TILES pairs; the kernel writes at most one
 * pair per 32 x 32 tile).  A stack of more than that many tiles,
 * n_img ceil(h/32) ceil(w/32), returns GS_EUNSUPPORTED before any launch.  The call makes no hipMalloc, hipFree or
 * other allocating call; the first call on a device looks up that device's
 * buffer address once.  Every call on one GPU shares its buffer: calls that
 * overlap on one GPU (streams or threads with no ordering between them) race
 * and their losses are undefined; calls ordered on one stream are safe.  The
 * buffer needs no clearing: a call writes every partial sum it reads. */
#define GS_LOSS_IMAGE_NOALLOC_TILES 262144
GS_API gs_status gs_loss_image_noalloc(const float *render, const float *measured, int32_t n_img,
                                       int32_t h, int32_t w, float lambda_ssim, float *loss_out,
                                       float *grad, hipStream_t stream);

/* 3D total variation of a block [nz][ny][nx] (Eq. 8 regularizer): the sum
 * over the three axes of the mean absolute forward difference.
 * loss_out (device, 1 float): the TV value (unweighted).
 * grad (device, may be NULL): weight * d TV / d volume (sign(0) = 0),
 * overwritten, or added to when accumulate != 0.  plan must not be NULL. */
GS_API gs_status gs_loss_tv(const float *volume, int32_t nx, int32_t ny, int32_t nz, float weight,
                     float *loss_out, float *grad, int32_t accumulate, gs_plan *plan,
                     hipStream_t stream);

/* Choose the projection's density scaling for later calls on this plan:
 * enable = 1 (default) renders the rectified density rho_hat = mu rho of
 * Eq. 7, mu = sqrt(2 pi |Sigma_tilde| / |Sigma_hat|); enable = 0 renders
 * rho_hat = rho, the 3DGS-style unrectified reading whose integration bias the
 * paper analyses (Sec. 3.2.1 "Integration bias"; the X-3DGS baseline of
 * Sec. 4.3).  gs_project_bwd differentiates whichever was chosen. */
GS_API gs_status gs_plan_set_rectify(gs_plan *plan, int32_t enable);

/* Per-Gaussian mean over the views of the rectification factor mu (views in
 * which the Gaussian is culled are left out; 0 if culled in all).  Dividing an
 * unrectified model's densities by it is the paper's correction of X-3DGS
 * before voxelization (Sec. 4.3).  mu_out: device [n] or NULL; density_out:
 * device [n] or NULL, receives density / mean mu (0 where the mean is 0).  At
 * least one of the two must be given (else GS_EINVAL).  The plan's view buffer
 * is reused, so the next projection call on the plan bins again. */
GS_API gs_status gs_project_mean_mu(const gs_gaussians *g, const gs_view *views, int32_t n_views,
                                    float *mu_out, float *density_out, gs_plan *plan,
                                    hipStream_t stream);

/* Stages of the launch sequences, for gs_plan_stage_times. */
typedef enum {
  GS_STAGE_PROJ_BIN = 0,     /* projection + rectification, tile histograms, scans */
  GS_STAGE_PROJ_SCATTER = 1, /* tile lists and backward slot offsets */
  GS_STAGE_RENDER_FWD = 2,   /* per-tile sum of rectified 2D Gaussians */
  GS_STAGE_RENDER_BWD = 3,   /* per-(tile, Gaussian) gradient moments */
  GS_STAGE_PROJ_CHAIN = 4,   /* per-Gaussian chain rule over views */
  GS_STAGE_VOX_BIN = 5,
  GS_STAGE_VOX_SCATTER = 6,
  GS_STAGE_VOX_FWD = 7,
  GS_STAGE_VOX_BWD = 8,
  GS_STAGE_VOX_CHAIN = 9,
  GS_STAGE_LOSS_IMAGE = 10,
  GS_STAGE_LOSS_TV = 11,
  GS_N_STAGES = 12
} gs_stage;

/* Enable (1) or disable (0) per-stage timing on a plan: each stage of each
 * later call is bracketed by two HIP events on the call's stream. */
GS_API gs_status gs_plan_set_timing(gs_plan *plan, int32_t enable);

/* Synchronize the plan's last stream and return, per stage, the summed
 * elapsed milliseconds (ms_sum, host [n]) and the number of timed launches
 * (count, host [n]) since the previous query; then reset.  n <= GS_N_STAGES. */
GS_API gs_status gs_plan_stage_times(gs_plan *plan, double *ms_sum, int64_t *count, int32_t n);

/* Thread-local message describing the last non-OK status ("" if none). */
GS_API const char *gs_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* GS_H */
