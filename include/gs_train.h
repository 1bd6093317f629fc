/*
 * gs_train.h - the optimisation loop around the rasterizer and voxelizer
 * (Sec. 3.3 "Optimization", Sec. 4.1 implementation details): densification
 * statistics, Adam with the exponential learning-rate decay, adaptive density
 * control, 3D evaluation metrics, and a trainer that runs the whole loop on
 * one stream.
 *
 * Readings of points the paper leaves to 3DGS:
 *   activations   mean and quaternion used as they are (the operators
 *                 normalise the quaternion); scale = exp(log_scale);
 *                 density = softplus(density_raw) = log(1 + exp(x)).
 *   Adam          beta1 0.9, beta2 0.999, eps 1e-15; one step counter shared
 *                 by all Gaussians; moments of new Gaussians start at zero.
 *   lr decay      lr(k) = lr0 * ratio^(k / iterations), k the 0-based iteration.
 *   statistics    per Gaussian, the sum over the views in which it is visible
 *                 (its cutoff ellipse's bounding box covers a pixel centre) of
 *                 |dL/dp_hat| in normalised device coordinates (detector
 *                 half-width and half-height = 1), and the number of those
 *                 views; the mean decides densification.
 *   densify       mean statistic >= grad_threshold: clone if the largest scale
 *                 is <= clone_max_scale, else split into two children at
 *                 p + R (s * z), z ~ N(0, I), with scales s / 1.6.  Both
 *                 resulting Gaussians get half the density (Sec. 3.3).  Any
 *                 resulting Gaussian with density < min_density is removed;
 *                 no Gaussian is removed for being large (Sec. 3.3).
 *   metrics       PSNR over the volume with data range max(gt); SSIM = mean
 *                 over the three axes of the mean 2D SSIM of the slices
 *                 normal to the axis (11x11 window, sigma 1.5, data range
 *                 max(gt), zero padding) (Sec. 4.1).
 *
 * All arrays are device memory owned by the caller unless stated otherwise.
 */
#ifndef GS_TRAIN_H
#define GS_TRAIN_H

#include "gs.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Densification statistics accumulated by gs_project_bwd_stats. */
typedef struct {
  float *grad_sum;   /* device [n]: += scale * sum of per-view NDC gradient norms */
  int32_t *visible;  /* device [n]: += number of views in which the Gaussian is visible */
  float scale;       /* multiplies the norms, e.g. the number of views whose mean loss
                        was differentiated, so that the statistic is per view */
} gs_grad_stats;

/* gs_project_bwd, and in the same pass the densification statistics above
 * (adds to stats->grad_sum and stats->visible, never clears them).
 * GS_EINVAL if stats or its arrays are NULL. */
GS_API gs_status gs_project_bwd_stats(const gs_gaussians *g, const gs_view *views, int32_t n_views,
                                      float cutoff, const float *grad_image, const gs_grads *grads,
                                      int32_t accumulate, const gs_grad_stats *stats,
                                      gs_plan *plan, hipStream_t stream);

/* Trainable state of up to `capacity` Gaussians, device SoA arrays.  The raw
 * arrays are what Adam updates; scale and density hold the activated values
 * that the rasterizer reads (with mean and quat, they form the gs_gaussians of
 * the model).  m_* and v_* are Adam's first and second moments, laid out like
 * the raw array of the same name. */
typedef struct {
  float *mean;         /* [capacity][3] */
  float *log_scale;    /* [capacity][3] */
  float *quat;         /* [capacity][4] */
  float *density_raw;  /* [capacity] */
  float *scale;        /* [capacity][3] = exp(log_scale) */
  float *density;      /* [capacity] = softplus(density_raw) */
  float *m_mean, *m_scale, *m_quat, *m_density;
  float *v_mean, *v_scale, *v_quat, *v_density;
} gs_params;

typedef struct {
  float lr_mean, lr_scale, lr_quat, lr_density;  /* this step's learning rates */
  int32_t step;                                  /* 1-based step count (bias correction) */
} gs_adam_config;

/* One Adam step on n Gaussians: grads are the gradients with respect to the
 * activated parameters (as gs_project_bwd gives them); the kernel applies the
 * activations' derivatives, updates moments and raw parameters, and rewrites
 * scale and density.  grads arrays must not alias the state.  No sync. */
GS_API gs_status gs_adam_step(const gs_params *p, int64_t n, const gs_grads *grads,
                              const gs_adam_config *cfg, hipStream_t stream);

/* Activated arrays from raw ones (scale = exp(log_scale), density =
 * softplus(density_raw)) for n Gaussians, e.g. after loading raw parameters. */
GS_API gs_status gs_params_activate(const gs_params *p, int64_t n, hipStream_t stream);

/* Raw arrays from activated ones (log_scale = log(scale), density_raw =
 * softplus^-1(density)); scale and density must be > 0. */
GS_API gs_status gs_params_from_activated(const gs_params *p, int64_t n, hipStream_t stream);

typedef struct {
  float grad_threshold;   /* mean statistic that triggers densification (5e-5, Sec. 4.1) */
  float clone_max_scale;  /* largest scale up to which a Gaussian is cloned, else split */
  float min_density;      /* resulting Gaussians below this density are removed */
  int32_t densify;        /* 0: only remove empty Gaussians */
} gs_densify_config;

/* n standard normal draws into out (device [n]), e.g. the split draws of
 * gs_densify: Philox4x32-10 (Salmon et al., SC 2011) with counter
 * (b, counter_lo, counter_hi, 0) and key (seed_lo, seed_hi) gives four words
 * for elements 4b .. 4b + 3; each word x becomes u = (x + 1/2) 2^-32 and the
 * pairs (u0, u1), (u2, u3) become sqrt(-2 ln u) (cos 2 pi v, sin 2 pi v)
 * (Box-Muller), evaluated in double and rounded.  No sync. */
GS_API gs_status gs_random_normals(uint64_t seed, uint64_t counter, int64_t n, float *out,
                                   hipStream_t stream);

/* Adaptive density control (Sec. 3.3) from src (n Gaussians) into dst
 * (capacity dst_capacity; dst must not overlap src).  Each source Gaussian
 * writes its 0, 1 or 2 results in source order: kept -> itself (same
 * moments); cloned -> itself with half density (same moments) then the copy
 * (zero moments); split -> two children (zero moments); removed -> nothing.
 * stats: grad_sum, visible [n] as accumulated by gs_project_bwd_stats.
 * normals: device [n][2][3] standard normal draws for the split children
 * (may be NULL when cfg->densify == 0).  action: device [n] or NULL, receives
 * 0 removed, 1 kept, 2 cloned, 3 split.  Decisions compare the FP32 raw
 * density with FP32 softplus^-1(min_density) (kept) or softplus^-1(2
 * min_density) (densified), the raw log-scales with FP32 log(clone_max_scale)
 * and the FP32 mean statistic grad_sum / visible with grad_threshold.
 * *n_out (host) receives the new count; if it exceeds dst_capacity, returns
 * GS_EOVERFLOW with *n_out set and dst untouched.  Synchronizes `stream`.
 * plan must not be NULL (holds the count scan). */
GS_API gs_status gs_densify(const gs_params *src, int64_t n, const gs_grad_stats *stats,
                            const float *normals, const gs_densify_config *cfg, gs_params *dst,
                            int64_t dst_capacity, int32_t *action, int64_t *n_out, gs_plan *plan,
                            hipStream_t stream);

/* PSNR and SSIM of a volume [nz][ny][nx] against the ground truth (Sec. 4.1,
 * readings above).  psnr and ssim are host doubles (either may be NULL).
 * GS_EINVAL if max(gt) <= 0.  Synchronizes `stream`; plan must not be NULL. */
GS_API gs_status gs_volume_metrics(const float *volume, const float *gt, int32_t nx, int32_t ny,
                                   int32_t nz, double *psnr, double *ssim, gs_plan *plan,
                                   hipStream_t stream);

/* ---- trainer: the loop of Sec. 3.3 / Sec. 4.1 on one stream ------------- */

typedef struct gs_trainer gs_trainer;

typedef struct {
  int32_t iterations;        /* length of the learning-rate schedule (30000) */
  int32_t views_per_iter;    /* views rendered per iteration (1) */
  float lr_mean, lr_density, lr_scale, lr_quat;  /* 2e-4, 1e-2, 5e-3, 1e-3 */
  float lr_final_ratio;      /* 0.1 */
  float lambda_ssim;         /* 0.25 */
  float lambda_tv;           /* 0.05 (0: no TV term) */
  int32_t tv_size;           /* D of the random TV block (32) */
  int32_t densify_from, densify_until, densify_interval;  /* 500, 15000, 100 */
  float grad_threshold;      /* 5e-5 */
  float clone_max_scale;     /* see gs_densify_config */
  float min_density;         /* see gs_densify_config */
  float cutoff;              /* Mahalanobis cutoff (3) */
  int32_t rectify;           /* 1: R^2-Gaussian; 0: the unrectified X-3DGS variant */
  uint64_t seed;             /* view order and TV blocks of gs_trainer_run (host generator);
                                split draws: gs_random_normals(seed, iteration index) */
} gs_train_config;

/* Fills the defaults of Sec. 4.1 (clone_max_scale 0.02, min_density 1e-4 and
 * cutoff 3 are readings). */
GS_API void gs_train_config_default(gs_train_config *cfg);

/* init: initial Gaussians (device, activated; copied).  measured: device
 * [n_views][h][w] log-space projections (kept by pointer, must outlive the
 * trainer).  views: host, copied.  grid: the reconstruction grid (the TV
 * block is a D^3 sub-grid of it at the same spacing).  Allocates its state
 * with hipMalloc and runs on a non-blocking stream of its own. */
GS_API gs_status gs_trainer_create(const gs_train_config *cfg, const gs_gaussians *init,
                                   const float *measured, const gs_view *views, int32_t n_views,
                                   const gs_grid *grid, gs_trainer **out);
GS_API void gs_trainer_destroy(gs_trainer *tr);

/* Runs `iters` iterations drawing views (a reshuffled stack, as 3DGS does)
 * and TV block offsets from the seeded host generator, and the split draws of
 * a densifying iteration k (1-based) as gs_random_normals(seed, k - 1).
 * losses: host [iters] or NULL, receives each iteration's total loss (Eq. 8).
 * Synchronizes at the end only (and at densification steps). */
GS_API gs_status gs_trainer_run(gs_trainer *tr, int32_t iters, float *losses);

/* One iteration with explicit draws: view_idx [views_per_iter] (host),
 * tv_offset[3] (host, voxel offset of the TV block in the grid), normals
 * (device [n][2][3] for the current count n, used only if this iteration
 * densifies; NULL otherwise).  loss: host, may be NULL (then no sync); with a
 * loss the call also checks the trainer's reserved plans (GS_EOVERFLOW if an
 * iteration's tile lists exceeded them). */
GS_API gs_status gs_trainer_step(gs_trainer *tr, const int32_t *view_idx, const int32_t *tv_offset,
                                 const float *normals, float *loss);

/* Current model: device pointers (activated parameters) valid until the next
 * trainer call; *iteration = iterations done. */
GS_API gs_status gs_trainer_model(gs_trainer *tr, gs_gaussians *out, int32_t *iteration);

/* Copies the current model (activated parameters) into caller device arrays
 * of the given capacity (mean [capacity][3], scale [capacity][3], quat
 * [capacity][4], density [capacity]); *n (host) receives the count.  Returns
 * GS_EOVERFLOW with *n set if the model does not fit.  Synchronizes. */
GS_API gs_status gs_trainer_export(gs_trainer *tr, int64_t capacity, float *mean, float *scale,
                                   float *quat, float *density, int64_t *n);

/* Current raw state (device pointers valid until the next trainer call) and
 * the densification statistics accumulated since the last densification. */
GS_API gs_status gs_trainer_state(gs_trainer *tr, gs_params *params, int64_t *n,
                                  gs_grad_stats *stats);

/* Voxelizes the model on grid (for the X-3DGS variant, densities divided by
 * their mean rectification factor over the training views first, Sec. 4.3)
 * into volume (device [nz][ny][nx]); with gt non-NULL also computes PSNR and
 * SSIM (host doubles, may be NULL).  Synchronizes. */
GS_API gs_status gs_trainer_evaluate(gs_trainer *tr, const gs_grid *grid, float *volume,
                                     const float *gt, double *psnr, double *ssim);

#ifdef __cplusplus
}
#endif

#endif /* GS_TRAIN_H */
