// Trainer: the optimisation loop of Sec. 3.3 / Sec. 4.1 on one HIP stream,
// built only on the public C ABI (gs.h, gs_train.h).  One iteration renders a
// batch of views, takes L1 + D-SSIM against the measured projections, adds
// the TV of a random D^3 block of the reconstruction grid, back-propagates
// both into the Gaussians (with densification statistics), applies Adam with
// the decayed learning rates, and every densify_interval iterations inside
// [densify_from, densify_until) runs the adaptive control into the second of
// two double-buffered parameter sets.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "../../include/gs_train.h"
#include "internal.h"

namespace {

// One parameter set: a single device allocation carved into the SoA arrays of
// gs_params (37 floats per Gaussian of capacity).
struct ParamSet {
  float *base = nullptr;
  int64_t cap = 0;
  gs_params p{};
};

constexpr int64_t kFloatsPerGaussian = 3 + 3 + 4 + 1 + 3 + 1 + 2 * (3 + 3 + 4 + 1);

void carve(ParamSet &s) {
  float *b = s.base;
  const int64_t c = s.cap;
  auto take = [&](int64_t k) {
    float *r = b;
    b += k * c;
    return r;
  };
  s.p.mean = take(3);
  s.p.log_scale = take(3);
  s.p.quat = take(4);
  s.p.density_raw = take(1);
  s.p.scale = take(3);
  s.p.density = take(1);
  s.p.m_mean = take(3);
  s.p.m_scale = take(3);
  s.p.m_quat = take(4);
  s.p.m_density = take(1);
  s.p.v_mean = take(3);
  s.p.v_scale = take(3);
  s.p.v_quat = take(4);
  s.p.v_density = take(1);
}

gs_status alloc_set(ParamSet &s, int64_t cap) {
  if (s.base) (void)hipFree(s.base);
  s.base = nullptr;
  s.cap = 0;
  if (hipMalloc(&s.base, sizeof(float) * kFloatsPerGaussian * (size_t)std::max<int64_t>(cap, 1)) !=
      hipSuccess) {
    (void)hipGetLastError();
    s.base = nullptr;
    return GS_ENOMEM;
  }
  s.cap = std::max<int64_t>(cap, 1);
  carve(s);
  return GS_OK;
}

template <class T> gs_status grow(T *&p, size_t &cap, size_t want) {
  if (cap >= want) return GS_OK;
  if (p) (void)hipFree(p);
  p = nullptr;
  cap = 0;
  want = std::max<size_t>(want, 1);
  if (hipMalloc((void **)&p, sizeof(T) * want) != hipSuccess) {
    (void)hipGetLastError();
    p = nullptr;
    return GS_ENOMEM;
  }
  cap = want;
  return GS_OK;
}

#define TR_TRY(x)                 \
  do {                            \
    gs_status _st = (x);          \
    if (_st != GS_OK) return _st; \
  } while (0)

gs_status invalid(const char *msg) {
  gsk::set_last_error(msg);
  return GS_EINVAL;
}

}  // namespace

struct gs_trainer {
  gs_train_config cfg{};
  hipStream_t stream = nullptr;
  gs_plan *proj = nullptr, *vox = nullptr, *loss = nullptr, *aux = nullptr;
  ParamSet sets[2];
  int cur = 0;
  int64_t n = 0;
  float *g_mean = nullptr, *g_scale = nullptr, *g_quat = nullptr, *g_dens = nullptr;
  size_t g_cap = 0, g_cap_s = 0, g_cap_q = 0, g_cap_d = 0;
  float *st_sum = nullptr;
  int32_t *st_vis = nullptr;
  size_t st_cap = 0, st_cap_v = 0;
  float *render = nullptr, *meas_batch = nullptr, *grad_img = nullptr;
  size_t render_cap = 0, meas_cap = 0, grad_cap = 0;
  float *tv_vol = nullptr, *tv_grad = nullptr;
  size_t tv_cap = 0, tv_grad_cap = 0;
  float *loss_dev = nullptr;
  size_t loss_cap = 0;
  float *normals = nullptr;
  size_t normals_cap = 0;
  float *dens_corr = nullptr;
  size_t dens_corr_cap = 0;
  const float *measured = nullptr;
  std::vector<gs_view> views;
  gs_grid grid{};
  int32_t iter = 0;
  std::mt19937_64 rng;
  std::vector<int32_t> stack;
  std::vector<gs_view> batch;
  // reserved plans (no allocation and no synchronization per iteration)
  bool reserved = false;
  int64_t res_gaussians = 0, res_proj_entries = 0, res_vox_entries = 0;
};

namespace {

gs_gaussians model_of(const gs_trainer *t) {
  const gs_params &p = t->sets[t->cur].p;
  gs_gaussians g{};
  g.n = t->n;
  g.mean = p.mean;
  g.scale = p.scale;
  g.quat = p.quat;
  g.density = p.density;
  return g;
}

gs_status ensure_per_gaussian(gs_trainer *t, int64_t n) {
  const size_t m = (size_t)std::max<int64_t>(n, 1);
  TR_TRY(grow(t->g_mean, t->g_cap, 3 * m));
  TR_TRY(grow(t->g_scale, t->g_cap_s, 3 * m));
  TR_TRY(grow(t->g_quat, t->g_cap_q, 4 * m));
  TR_TRY(grow(t->g_dens, t->g_cap_d, m));
  TR_TRY(grow(t->st_sum, t->st_cap, m));
  TR_TRY(grow(t->st_vis, t->st_cap_v, m));
  return GS_OK;
}

gs_status clear_stats(gs_trainer *t) {
  if (t->n == 0) return GS_OK;
  if (hipMemsetAsync(t->st_sum, 0, sizeof(float) * (size_t)t->n, t->stream) != hipSuccess ||
      hipMemsetAsync(t->st_vis, 0, sizeof(int32_t) * (size_t)t->n, t->stream) != hipSuccess)
    return GS_EHIP;
  return GS_OK;
}

// (Re)reserves the projection, voxel and loss plans for the current capacity
// and 3x the given entry counts.
gs_status reserve_plans(gs_trainer *t, int64_t proj_entries, int64_t vox_entries) {
  const gs_train_config &c = t->cfg;
  const int64_t cap = std::max(t->sets[0].cap, t->sets[1].cap);
  const int D = c.tv_size;
  const bool tv = c.lambda_tv > 0.f && D > 0;
  gs_reserve r{};
  r.max_gaussians = cap;
  r.max_views = c.views_per_iter;
  r.width = t->views[0].width;
  r.height = t->views[0].height;
  r.max_proj_entries = std::min<int64_t>(3 * std::max<int64_t>(proj_entries, 1024), 0xfffffffeLL);
  TR_TRY(gs_plan_reserve(t->proj, &r, t->stream));
  if (tv) {
    gs_reserve v{};
    v.max_gaussians = cap;
    v.nx = std::min(D, t->grid.nx);
    v.ny = std::min(D, t->grid.ny);
    v.nz = std::min(D, t->grid.nz);
    // the random block's entries vary with its position; a Gaussian meets at
    // most every 8^3 tile of the block, which bounds them for any position
    const int64_t tiles = (int64_t)((v.nx + 7) / 8) * ((v.ny + 7) / 8) * ((v.nz + 7) / 8);
    v.max_vox_entries = std::min<int64_t>(std::max<int64_t>(cap * tiles, 1024), 0xfffffffeLL);
    (void)vox_entries;
    TR_TRY(gs_plan_reserve(t->vox, &v, t->stream));
  }
  gs_reserve l{};
  l.max_views = c.views_per_iter;
  l.width = t->views[0].width;
  l.height = t->views[0].height;
  l.max_tv_voxels = tv ? (int64_t)D * D * D : 0;
  TR_TRY(gs_plan_reserve(t->loss, &l, t->stream));
  t->reserved = true;
  t->res_gaussians = cap;
  t->res_proj_entries = r.max_proj_entries;
  t->res_vox_entries = 0;  // bounded by construction (see above)
  return GS_OK;
}

// At a synchronization point: grow the reservation when the largest need
// since the last check passed half of it, exceeded it, or the parameter
// capacity grew, then fail if an iteration exceeded the reserved tile lists.
// Such iterations changed no parameter (their Adam steps are guarded on the
// plans' overflow records), and the grown reservation lets a new run go on.
gs_status check_plans(gs_trainer *t) {
  if (!t->reserved) return GS_OK;
  int64_t pe = 0, ve = 0, unused = 0;
  const gs_status sp = gs_plan_check(t->proj, &pe, &unused);
  if (sp != GS_OK && sp != GS_EOVERFLOW) return sp;
  gs_status sv = GS_OK;
  if (t->cfg.lambda_tv > 0.f && t->cfg.tv_size > 0) {
    sv = gs_plan_check(t->vox, &unused, &ve);
    if (sv != GS_OK && sv != GS_EOVERFLOW) return sv;
  }
  const int64_t cap = std::max(t->sets[0].cap, t->sets[1].cap);
  (void)ve;
  const bool over = sp == GS_EOVERFLOW || sv == GS_EOVERFLOW;
  if (over || 2 * pe > t->res_proj_entries || cap > t->res_gaussians)
    TR_TRY(reserve_plans(t, std::max(pe, t->res_proj_entries / 3), 0));
  if (over) {
    gsk::set_last_error("iterations needed more tile entries than reserved: their parameter "
                        "updates were skipped and the reservation has grown; run again");
    return GS_EOVERFLOW;
  }
  return GS_OK;
}

bool densify_due(const gs_train_config &c, int32_t it1) {
  return c.densify_interval > 0 && it1 > c.densify_from && it1 < c.densify_until &&
         it1 % c.densify_interval == 0;
}

gs_status densify(gs_trainer *t, const float *normals) {
  const gs_train_config &c = t->cfg;
  gs_densify_config dc{c.grad_threshold, c.clone_max_scale, c.min_density, 1};
  gs_grad_stats st{t->st_sum, t->st_vis, 1.f};
  ParamSet &src = t->sets[t->cur], &dst = t->sets[1 - t->cur];
  int64_t n_new = 0;
  gs_status s = gs_densify(&src.p, t->n, &st, normals, &dc, &dst.p, dst.cap, nullptr, &n_new,
                           t->aux, t->stream);
  if (s == GS_EOVERFLOW) {
    TR_TRY(alloc_set(dst, n_new + n_new / 2 + 1024));
    s = gs_densify(&src.p, t->n, &st, normals, &dc, &dst.p, dst.cap, nullptr, &n_new, t->aux,
                   t->stream);
  }
  TR_TRY(s);
  t->cur = 1 - t->cur;
  t->n = n_new;
  TR_TRY(ensure_per_gaussian(t, n_new));
  return clear_stats(t);
}

gs_status step(gs_trainer *t, const int32_t *view_idx, const int32_t *tv_offset,
               const float *normals, float *loss_slot) {
  const gs_train_config &c = t->cfg;
  const int B = c.views_per_iter;
  const int W = t->views[0].width, H = t->views[0].height;
  const size_t img = (size_t)W * H;
  if (densify_due(c, t->iter + 1) && !normals)
    return invalid("this iteration densifies: the split draws (normals) are required");
  t->batch.resize(B);
  for (int b = 0; b < B; ++b) {
    if (view_idx[b] < 0 || view_idx[b] >= (int32_t)t->views.size())
      return invalid("view index out of range");
    t->batch[b] = t->views[view_idx[b]];
  }
  const int D = c.tv_size;
  const bool tv = c.lambda_tv > 0.f && D > 0;
  gs_grid block{};
  if (tv) {
    const int dims[3] = {t->grid.nx, t->grid.ny, t->grid.nz};
    int bd[3];
    for (int k = 0; k < 3; ++k) {
      bd[k] = std::min(D, dims[k]);
      if (tv_offset[k] < 0 || tv_offset[k] > dims[k] - bd[k])
        return invalid("TV block offset outside the grid");
      block.origin[k] = t->grid.origin[k] + (float)tv_offset[k] * t->grid.spacing[k];
      block.spacing[k] = t->grid.spacing[k];
    }
    block.nx = bd[0];
    block.ny = bd[1];
    block.nz = bd[2];
  }
  TR_TRY(grow(t->render, t->render_cap, img * B));
  TR_TRY(grow(t->grad_img, t->grad_cap, img * B));
  const float *meas = t->measured + (size_t)view_idx[0] * img;
  if (B > 1) {
    TR_TRY(grow(t->meas_batch, t->meas_cap, img * B));
    for (int b = 0; b < B; ++b)
      if (hipMemcpyAsync(t->meas_batch + b * img, t->measured + (size_t)view_idx[b] * img,
                         sizeof(float) * img, hipMemcpyDeviceToDevice, t->stream) != hipSuccess)
        return GS_EHIP;
    meas = t->meas_batch;
  }
  gs_gaussians g = model_of(t);
  TR_TRY(gs_project_fwd(&g, t->batch.data(), B, c.cutoff, t->render, t->proj, t->stream));
  TR_TRY(gs_loss_image(t->render, meas, B, H, W, c.lambda_ssim, loss_slot, t->grad_img, t->loss,
                       t->stream));
  if (tv) {
    const size_t nv = (size_t)block.nx * block.ny * block.nz;
    TR_TRY(grow(t->tv_vol, t->tv_cap, nv));
    TR_TRY(grow(t->tv_grad, t->tv_grad_cap, nv));
    TR_TRY(gs_voxelize_fwd(&g, &block, c.cutoff, t->tv_vol, t->vox, t->stream));
    TR_TRY(gs_loss_tv(t->tv_vol, block.nx, block.ny, block.nz, c.lambda_tv, loss_slot + 3,
                      t->tv_grad, 0, t->loss, t->stream));
  } else if (hipMemsetAsync(loss_slot + 3, 0, sizeof(float), t->stream) != hipSuccess) {
    return GS_EHIP;
  }
  gs_grads gr{t->g_mean, t->g_scale, t->g_quat, t->g_dens};
  const int32_t it1 = t->iter + 1;
  if (it1 < c.densify_until) {
    gs_grad_stats st{t->st_sum, t->st_vis, (float)B};
    TR_TRY(gs_project_bwd_stats(&g, t->batch.data(), B, c.cutoff, t->grad_img, &gr, 0, &st,
                                t->proj, t->stream));
  } else {
    TR_TRY(gs_project_bwd(&g, t->batch.data(), B, c.cutoff, t->grad_img, &gr, 0, t->proj,
                          t->stream));
  }
  if (tv)
    TR_TRY(gs_voxelize_bwd(&g, &block, c.cutoff, t->tv_grad, &gr, 1, t->vox, t->stream));
  const double f = std::pow((double)c.lr_final_ratio, (double)t->iter / (double)c.iterations);
  gs_adam_config ac{(float)(c.lr_mean * f), (float)(c.lr_scale * f), (float)(c.lr_quat * f),
                    (float)(c.lr_density * f), it1};
  TR_TRY(gsk::adam_step_guarded(&t->sets[t->cur].p, t->n, &gr, &ac, t->reserved ? t->proj : nullptr,
                                 t->reserved && tv ? t->vox : nullptr, t->stream));
  t->iter = it1;
  if (densify_due(c, it1)) {
    TR_TRY(densify(t, normals));
    TR_TRY(check_plans(t));
  }
  if (!t->reserved) {
    // the first iteration ran with allocating plans: size the reservation
    // from its tile-list entries
    int64_t pe = 0, ve = 0;
    TR_TRY(gs_plan_status(t->proj, nullptr, &pe));
    if (tv) TR_TRY(gs_plan_status(t->vox, nullptr, &ve));
    TR_TRY(reserve_plans(t, pe, ve));
  }
  return GS_OK;
}

}  // namespace

extern "C" {

void gs_train_config_default(gs_train_config *c) {
  if (!c) return;
  std::memset(c, 0, sizeof(*c));
  c->iterations = 30000;
  c->views_per_iter = 1;
  c->lr_mean = 2e-4f;
  c->lr_density = 1e-2f;
  c->lr_scale = 5e-3f;
  c->lr_quat = 1e-3f;
  c->lr_final_ratio = 0.1f;
  c->lambda_ssim = 0.25f;
  c->lambda_tv = 0.05f;
  c->tv_size = 32;
  c->densify_from = 500;
  c->densify_until = 15000;
  c->densify_interval = 100;
  c->grad_threshold = 5e-5f;
  c->clone_max_scale = 0.02f;
  c->min_density = 1e-4f;
  c->cutoff = 3.f;
  c->rectify = 1;
  c->seed = 0;
}

void gs_trainer_destroy(gs_trainer *t) {
  if (!t) return;
  if (t->stream) (void)hipStreamSynchronize(t->stream);
  gs_plan_destroy(t->proj);
  gs_plan_destroy(t->vox);
  gs_plan_destroy(t->loss);
  gs_plan_destroy(t->aux);
  for (auto &s : t->sets)
    if (s.base) (void)hipFree(s.base);
  void *bufs[] = {t->g_mean, t->g_scale, t->g_quat, t->g_dens, t->st_sum, t->st_vis,
                  t->render, t->meas_batch, t->grad_img, t->tv_vol, t->tv_grad, t->loss_dev,
                  t->normals, t->dens_corr};
  for (void *b : bufs)
    if (b) (void)hipFree(b);
  if (t->stream) (void)hipStreamDestroy(t->stream);
  delete t;
}

gs_status gs_trainer_create(const gs_train_config *cfg, const gs_gaussians *init,
                            const float *measured, const gs_view *views, int32_t n_views,
                            const gs_grid *grid, gs_trainer **out) {
  if (!out) return invalid("out is NULL");
  *out = nullptr;
  if (!cfg || !init || !measured || !views || n_views < 1 || !grid)
    return invalid("NULL argument or no views");
  if (cfg->iterations < 1 || cfg->views_per_iter < 1 || cfg->views_per_iter > n_views ||
      cfg->tv_size < 0 || !(cfg->cutoff > 0.f) || !(cfg->lr_final_ratio > 0.f) ||
      cfg->densify_interval < 0)
    return invalid("invalid training configuration");
  if (init->n < 0 || (init->n > 0 && (!init->mean || !init->scale || !init->quat || !init->density)))
    return invalid("initial Gaussians incomplete");
  for (int i = 1; i < n_views; ++i)
    if (views[i].width != views[0].width || views[i].height != views[0].height)
      return invalid("views differ in detector size");
  if (grid->nx < 1 || grid->ny < 1 || grid->nz < 1) return invalid("grid size must be >= 1");
  gs_trainer *t = new (std::nothrow) gs_trainer();
  if (!t) return GS_ENOMEM;
  t->cfg = *cfg;
  t->measured = measured;
  t->views.assign(views, views + n_views);
  t->grid = *grid;
  t->rng.seed(cfg->seed);
  gs_status st = GS_OK;
  if (hipStreamCreateWithFlags(&t->stream, hipStreamNonBlocking) != hipSuccess) st = GS_EHIP;
  gs_plan **plans[] = {&t->proj, &t->vox, &t->loss, &t->aux};
  for (gs_plan **pp : plans)
    if (st == GS_OK) st = gs_plan_create(nullptr, nullptr, nullptr, pp);
  if (st == GS_OK) st = gs_plan_set_rectify(t->proj, cfg->rectify ? 1 : 0);
  t->n = init->n;
  if (st == GS_OK) st = alloc_set(t->sets[0], init->n * 2 + 1024);
  if (st == GS_OK) st = alloc_set(t->sets[1], init->n * 2 + 1024);
  if (st == GS_OK) st = ensure_per_gaussian(t, init->n);
  if (st == GS_OK && init->n > 0) {
    gs_params &p = t->sets[0].p;
    const size_t n = (size_t)init->n;
    if (hipMemcpyAsync(p.mean, init->mean, 12 * n, hipMemcpyDeviceToDevice, t->stream) != hipSuccess ||
        hipMemcpyAsync(p.scale, init->scale, 12 * n, hipMemcpyDeviceToDevice, t->stream) != hipSuccess ||
        hipMemcpyAsync(p.quat, init->quat, 16 * n, hipMemcpyDeviceToDevice, t->stream) != hipSuccess ||
        hipMemcpyAsync(p.density, init->density, 4 * n, hipMemcpyDeviceToDevice, t->stream) != hipSuccess ||
        hipMemsetAsync(p.m_mean, 0, sizeof(float) * 22 * (size_t)t->sets[0].cap, t->stream) != hipSuccess)
      st = GS_EHIP;
    if (st == GS_OK) st = gs_params_from_activated(&p, init->n, t->stream);
    if (st == GS_OK) st = clear_stats(t);
  }
  if (st == GS_OK && hipStreamSynchronize(t->stream) != hipSuccess) st = GS_EHIP;
  if (st != GS_OK) {
    gs_trainer_destroy(t);
    return st;
  }
  *out = t;
  return GS_OK;
}

gs_status gs_trainer_step(gs_trainer *t, const int32_t *view_idx, const int32_t *tv_offset,
                          const float *normals, float *loss) {
  if (!t || !view_idx || (!tv_offset && t->cfg.lambda_tv > 0.f && t->cfg.tv_size > 0))
    return GS_EINVAL;
  TR_TRY(grow(t->loss_dev, t->loss_cap, 4));
  const int32_t zero3[3] = {0, 0, 0};
  const gs_status st = step(t, view_idx, tv_offset ? tv_offset : zero3, normals, t->loss_dev);
  if (st == GS_EOVERFLOW) {  // a plan refused the call: grow the reservation and report
    const gs_status c = check_plans(t);
    return c == GS_OK ? GS_EOVERFLOW : c;
  }
  TR_TRY(st);
  if (loss) {
    float h[4];
    if (hipMemcpyAsync(h, t->loss_dev, sizeof(h), hipMemcpyDeviceToHost, t->stream) != hipSuccess ||
        hipStreamSynchronize(t->stream) != hipSuccess)
      return GS_EHIP;
    *loss = h[0] + t->cfg.lambda_tv * h[3];
    TR_TRY(check_plans(t));  // synchronized anyway: report any reservation overflow
  }
  return GS_OK;
}

gs_status gs_trainer_run(gs_trainer *t, int32_t iters, float *losses) {
  if (!t || iters < 0) return GS_EINVAL;
  if (iters == 0) return GS_OK;
  const gs_train_config &c = t->cfg;
  TR_TRY(grow(t->loss_dev, t->loss_cap, 4 * (size_t)iters));
  std::vector<int32_t> idx(c.views_per_iter);
  for (int32_t k = 0; k < iters; ++k) {
    for (int b = 0; b < c.views_per_iter; ++b) {
      if (t->stack.empty())
        for (int v = (int)t->views.size() - 1; v >= 0; --v) t->stack.push_back(v);
      std::uniform_int_distribution<size_t> pick(0, t->stack.size() - 1);
      const size_t j = pick(t->rng);
      idx[b] = t->stack[j];
      t->stack.erase(t->stack.begin() + (int64_t)j);
    }
    int32_t off[3] = {0, 0, 0};
    const int dims[3] = {t->grid.nx, t->grid.ny, t->grid.nz};
    for (int a = 0; a < 3; ++a) {
      std::uniform_int_distribution<int> o(0, std::max(0, dims[a] - c.tv_size));
      off[a] = o(t->rng);
    }
    const float *nrm = nullptr;
    if (densify_due(c, t->iter + 1)) {
      // split draws on the device: counter = index of this densification
      const size_t nz = 6 * (size_t)std::max<int64_t>(t->n, 1);
      TR_TRY(grow(t->normals, t->normals_cap, nz));
      TR_TRY(gs_random_normals(c.seed, (uint64_t)t->iter, (int64_t)nz, t->normals, t->stream));
      nrm = t->normals;
    }
    const gs_status st = step(t, idx.data(), off, nrm, t->loss_dev + 4 * (size_t)k);
    if (st == GS_EOVERFLOW) {  // a plan refused the call: grow the reservation and report
      const gs_status c = check_plans(t);
      return c == GS_OK ? GS_EOVERFLOW : c;
    }
    TR_TRY(st);
  }
  TR_TRY(check_plans(t));
  if (losses) {
    std::vector<float> h(4 * (size_t)iters);
    if (hipMemcpyAsync(h.data(), t->loss_dev, sizeof(float) * h.size(), hipMemcpyDeviceToHost,
                       t->stream) != hipSuccess)
      return GS_EHIP;
    if (hipStreamSynchronize(t->stream) != hipSuccess) return GS_EHIP;
    for (int32_t k = 0; k < iters; ++k) losses[k] = h[4 * k] + c.lambda_tv * h[4 * k + 3];
  } else if (hipStreamSynchronize(t->stream) != hipSuccess) {
    return GS_EHIP;
  }
  return GS_OK;
}

gs_status gs_trainer_model(gs_trainer *t, gs_gaussians *out, int32_t *iteration) {
  if (!t || !out) return GS_EINVAL;
  *out = model_of(t);
  if (iteration) *iteration = t->iter;
  return GS_OK;
}

gs_status gs_trainer_export(gs_trainer *t, int64_t capacity, float *mean, float *scale, float *quat,
                            float *density, int64_t *n) {
  if (!t || !n || capacity < 0) return GS_EINVAL;
  *n = t->n;
  if (t->n > capacity) return GS_EOVERFLOW;
  if (t->n == 0) return GS_OK;
  if (!mean || !scale || !quat || !density) return GS_EINVAL;
  const gs_params &p = t->sets[t->cur].p;
  const size_t m = (size_t)t->n;
  if (hipMemcpyAsync(mean, p.mean, 12 * m, hipMemcpyDeviceToDevice, t->stream) != hipSuccess ||
      hipMemcpyAsync(scale, p.scale, 12 * m, hipMemcpyDeviceToDevice, t->stream) != hipSuccess ||
      hipMemcpyAsync(quat, p.quat, 16 * m, hipMemcpyDeviceToDevice, t->stream) != hipSuccess ||
      hipMemcpyAsync(density, p.density, 4 * m, hipMemcpyDeviceToDevice, t->stream) != hipSuccess)
    return GS_EHIP;
  return hipStreamSynchronize(t->stream) == hipSuccess ? GS_OK : GS_EHIP;
}

gs_status gs_trainer_state(gs_trainer *t, gs_params *params, int64_t *n, gs_grad_stats *stats) {
  if (!t) return GS_EINVAL;
  if (params) *params = t->sets[t->cur].p;
  if (n) *n = t->n;
  if (stats) *stats = gs_grad_stats{t->st_sum, t->st_vis, 1.f};
  return GS_OK;
}

gs_status gs_trainer_evaluate(gs_trainer *t, const gs_grid *grid, float *volume, const float *gt,
                              double *psnr, double *ssim) {
  if (!t || !grid || !volume) return GS_EINVAL;
  gs_gaussians g = model_of(t);
  if (!t->cfg.rectify && g.n > 0) {
    TR_TRY(grow(t->dens_corr, t->dens_corr_cap, (size_t)g.n));
    TR_TRY(gs_project_mean_mu(&g, t->views.data(), (int32_t)t->views.size(), nullptr, t->dens_corr,
                              t->aux, t->stream));
    g.density = t->dens_corr;
  }
  TR_TRY(gs_voxelize_fwd(&g, grid, t->cfg.cutoff, volume, t->aux, t->stream));
  if (gt)
    TR_TRY(gs_volume_metrics(volume, gt, grid->nx, grid->ny, grid->nz, psnr, ssim, t->aux,
                             t->stream));
  return hipStreamSynchronize(t->stream) == hipSuccess ? GS_OK : GS_EHIP;
}

}  // extern "C"
