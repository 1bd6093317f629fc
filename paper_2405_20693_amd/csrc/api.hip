// C ABI of the HIP path: argument validation, plan workspace and the launch
// sequences of the projection, voxelization and loss entry points.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/gs.h"
#include "../../include/gs_train.h"
#include "internal.h"

using namespace gsk;

namespace {

thread_local std::string g_err;

gs_status fail(gs_status st, const std::string &msg) {
  g_err = msg;
  return st;
}

#define GS_TRY(x)                   \
  do {                              \
    gs_status _st = (x);            \
    if (_st != GS_OK) return _st;   \
  } while (0)

struct Buf {
  void *p = nullptr;
  size_t cap = 0;
};

struct ProjKey {
  const float *mean = nullptr, *scale = nullptr, *quat = nullptr, *dens = nullptr;
  int64_t n = -1;
  float cutoff = 0.f;
  std::vector<gs_view> views;
};

struct VoxKey {
  const float *mean = nullptr, *scale = nullptr, *quat = nullptr, *dens = nullptr;
  int64_t n = -1;
  float cutoff = 0.f;
  gs_grid grid{};
};

}  // namespace

struct gs_plan {
  gs_alloc_fn alloc = nullptr;
  gs_free_fn free_fn = nullptr;
  void *ctx = nullptr;
  hipStream_t last_stream = nullptr;
  bool used = false;
  // projection
  Buf p_views, p_rec, p_hist, p_tile_total, p_tile_start, p_chunk_cnt, p_chunk_start, p_offsets,
      p_list, p_slots, p_totals, p_part, p_scan_tmp, p_fpart;
  // voxelization
  Buf v_rec, v_count, v_offsets, v_scan_tmp, v_hist, v_tile_total, v_tile_start, v_list, v_slots,
      v_totals, v_fpart;
  // losses
  Buf l_coef, l_part;
  // adaptive control and metrics
  Buf d_action, d_count, d_offsets, d_scan_tmp, d_totals, m_sse, m_max, m_out, m_stack, m_loss;
  Buf skipped;  // control words, unsigned long long [8] (layout in internal.h)
  // host side: a ring of pinned staging buffers for per-view constants, so
  // that an upload waits only for the copy issued kStageRing uploads earlier
  static constexpr int kStageRing = 4;
  void *stage[kStageRing] = {};
  size_t stage_cap[kStageRing] = {};
  hipEvent_t stage_done[kStageRing] = {};
  bool stage_pending[kStageRing] = {};
  int stage_next = 0;
  std::vector<gs_view> up_views;     // the views p_views holds
  std::vector<ViewSet> up_sets;      // and their Gaussian sets (multi-model calls; else empty)
  bool up_valid = false;
  unsigned long long *readback = nullptr;  // pinned, 4 entries
  // reserved mode: no allocation and no synchronization in the operator calls
  bool reserved = false;
  // set by a scatter kernel whose call needed more entries than reserved
  // (pinned, mapped, coherent host memory: the host reads it without any
  // copy or synchronization); cleared by gs_plan_check
  unsigned int *ovf_flag = nullptr, *ovf_flag_dev = nullptr;
  gs_reserve res{};
  // saved forward state
  bool p_valid = false, v_valid = false;
  ProjKey pkey;
  VoxKey vkey;
  ProjArgs pargs{};
  VoxArgs vargs{};
  uint64_t p_entries = 0, v_entries = 0;
  // method option: rectified (R^2-Gaussian) or unrectified (X-3DGS) projection
  int rectify = 1;
  // per-stage timing
  bool timing = false;
  struct Timed {
    int stage;
    hipEvent_t a, b;
  };
  std::vector<Timed> timed;
  std::vector<hipEvent_t> event_pool;
};

namespace {

hipEvent_t pooled_event(gs_plan *pl) {
  if (!pl->event_pool.empty()) {
    hipEvent_t e = pl->event_pool.back();
    pl->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Brackets one stage with two events when the plan times its launches.
struct StageTimer {
  gs_plan *pl;
  hipStream_t s;
  int stage;
  hipEvent_t a = nullptr;
  StageTimer(gs_plan *p, int st, hipStream_t str) : pl(p), s(str), stage(st) {
    if (pl->timing) {
      a = pooled_event(pl);
      if (a) (void)hipEventRecord(a, s);
    }
  }
  void stop() {
    if (!a) return;
    hipEvent_t b = pooled_event(pl);
    if (b) {
      (void)hipEventRecord(b, s);
      pl->timed.push_back({stage, a, b});
    } else {
      pl->event_pool.push_back(a);
    }
    a = nullptr;
  }
  ~StageTimer() { stop(); }
};

gs_status sync_stream(gs_plan *pl, hipStream_t s) {
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(GS_EHIP, std::string("hipStreamSynchronize: ") + hipGetErrorString(e));
  return GS_OK;
}

void release(gs_plan *pl, Buf &b) {
  if (!b.p) return;
  if (pl->free_fn)
    pl->free_fn(b.p, pl->ctx);
  else
    (void)hipFree(b.p);
  b.p = nullptr;
  b.cap = 0;
}

// Grow-only workspace buffer.  Growing synchronizes `s` first so that no
// queued kernel still uses the old buffer.  A buffer grows by a quarter more
// than asked, unless `exact` (reservations).
gs_status ensure(gs_plan *pl, Buf &b, size_t bytes, hipStream_t s, bool exact = false) {
  if (bytes == 0) bytes = 256;
  if (b.cap >= bytes) return GS_OK;
  if (pl->reserved) return fail(GS_EINVAL, "the call exceeds the plan's reservation");
  if (b.p) {
    gs_status st = sync_stream(pl, s);
    if (st != GS_OK) return st;
    release(pl, b);
  }
  size_t want = exact ? bytes : bytes + bytes / 4;
  want = (want + 255) & ~(size_t)255;
  void *p = nullptr;
  if (pl->alloc) {
    p = pl->alloc(want, pl->ctx);
  } else if (hipMalloc(&p, want) != hipSuccess) {
    (void)hipGetLastError();
    p = nullptr;
  }
  if (!p) return fail(GS_ENOMEM, "workspace allocation of " + std::to_string(want) + " bytes failed");
  b.p = p;
  b.cap = want;
  return GS_OK;
}

// Skipped-Gaussian counters: the binning kernels add to the running counter
// of their operator (0 projection, 1 voxelization) and the scatter kernel of
// the same call moves it to the last-call slot (2, 3) and clears it, so no
// fill is needed per call.  All four start at zero.
gs_status ensure_skipped(gs_plan *pl, hipStream_t s) {
  if (pl->skipped.p) return GS_OK;
  GS_TRY(ensure(pl, pl->skipped, 64, s));
  if (hipMemsetAsync(pl->skipped.p, 0, 64, s) != hipSuccess) return fail(GS_EHIP, "hipMemsetAsync");
  return GS_OK;
}

// Clears a running counter when a call stops between binning and scatter.
gs_status clear_running_skipped(gs_plan *pl, int which, hipStream_t s) {
  if (hipMemsetAsync(reinterpret_cast<unsigned long long *>(pl->skipped.p) + which, 0, 8, s) !=
      hipSuccess)
    return fail(GS_EHIP, "hipMemsetAsync");
  return GS_OK;
}

gs_status check_launch(const char *what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(GS_EHIP, std::string(what) + ": " + hipGetErrorString(e));
  return GS_OK;
}


template <class T> T *P(Buf &b) { return reinterpret_cast<T *>(b.p); }

bool finite_pos(float x) { return std::isfinite(x) && x > 0.f; }

gs_status check_gaussians(const gs_gaussians *g) {
  if (!g) return fail(GS_EINVAL, "gaussians is NULL");
  if (g->n < 0) return fail(GS_EINVAL, "gaussians->n < 0");
  if (g->n > 0x7fffffffLL) return fail(GS_EUNSUPPORTED, "more than 2^31-1 Gaussians");
  if (g->n > 0 && (!g->mean || !g->scale || !g->quat || !g->density))
    return fail(GS_EINVAL, "a Gaussian array pointer is NULL");
  return GS_OK;
}

gs_status check_cutoff(float cutoff) {
  if (!(cutoff > 0.f)) return fail(GS_EINVAL, "cutoff must be > 0 (INFINITY for none)");
  return GS_OK;
}

gs_status check_views(const gs_view *views, int32_t n_views) {
  if (!views) return fail(GS_EINVAL, "views is NULL");
  if (n_views < 1) return fail(GS_EINVAL, "n_views < 1");
  const int w = views[0].width, h = views[0].height;
  for (int i = 0; i < n_views; ++i) {
    const gs_view &v = views[i];
    const std::string at = " (view " + std::to_string(i) + ")";
    if (v.beam != GS_PARALLEL && v.beam != GS_CONE) return fail(GS_EINVAL, "unknown beam" + at);
    if (v.width < 1 || v.height < 1 || v.width > 16384 || v.height > 16384)
      return fail(GS_EINVAL, "detector size out of 1..16384" + at);
    if (v.width != w || v.height != h) return fail(GS_EINVAL, "views differ in detector size" + at);
    if (!finite_pos(v.pitch_u) || !finite_pos(v.pitch_v)) return fail(GS_EINVAL, "pitch must be > 0" + at);
    if (!std::isfinite(v.off_u) || !std::isfinite(v.off_v)) return fail(GS_EINVAL, "offset not finite" + at);
    for (int k = 0; k < 9; ++k)
      if (!std::isfinite(v.rot[k])) return fail(GS_EINVAL, "rotation not finite" + at);
    if (v.beam == GS_CONE) {
      if (!finite_pos(v.src_obj) || !std::isfinite(v.src_det) || !(v.src_det > v.src_obj))
        return fail(GS_EINVAL, "cone beam needs 0 < src_obj < src_det" + at);
    }
  }
  return GS_OK;
}

gs_status check_grid(const gs_grid *grid) {
  if (!grid) return fail(GS_EINVAL, "grid is NULL");
  if (grid->nx < 1 || grid->ny < 1 || grid->nz < 1 || grid->nx > 16384 || grid->ny > 16384 ||
      grid->nz > 16384)
    return fail(GS_EINVAL, "grid size out of 1..16384");
  // the voxel binning keeps one z-layer of 8^3 tiles in LDS
  if ((int64_t)((grid->nx + kVTile - 1) / kVTile) * ((grid->ny + kVTile - 1) / kVTile) >
      kMaxTilesPerGroup)
    return fail(GS_EUNSUPPORTED, "grid plane has more than 16384 tiles");
  for (int k = 0; k < 3; ++k) {
    if (!finite_pos(grid->spacing[k])) return fail(GS_EINVAL, "grid spacing must be > 0");
    if (!std::isfinite(grid->origin[k])) return fail(GS_EINVAL, "grid origin not finite");
  }
  return GS_OK;
}

DevView make_dev_view(const gs_view &v) {
  DevView d{};
  for (int k = 0; k < 9; ++k) d.W[k] = v.rot[k];
  d.L_SO = v.src_obj;
  d.L_SD = v.src_det;
  d.hu = v.pitch_u;
  d.hv = v.pitch_v;
  d.inv_hu = (float)(1.0 / (double)v.pitch_u);
  d.inv_hv = (float)(1.0 / (double)v.pitch_v);
  d.cu = (float)(0.5 * v.width - 0.5 - (double)v.off_u / (double)v.pitch_u);
  d.cv = (float)(0.5 * v.height - 0.5 - (double)v.off_v / (double)v.pitch_v);
  d.beam = v.beam;
  return d;
}

void cutoff_consts(float cutoff, float &kappa, float &thr, float &qmax) {
  kappa = cutoff;
  if (std::isinf(cutoff)) {
    thr = -INFINITY;
    qmax = INFINITY;
  } else {
    double q = 0.5 * 1.4426950408889634 * (double)cutoff * (double)cutoff;
    thr = (float)(-q);
    qmax = (float)(q * (1.0 + 1e-5));
  }
}

// Uploads per-view constants (and, for a multi-model call, the views'
// Gaussian sets after them) through the pinned staging ring, unless p_views
// already holds exactly these.
gs_status upload_views(gs_plan *pl, const gs_view *views, int32_t nv, hipStream_t s,
                       const ViewSet *sets = nullptr) {
  const size_t vbytes = sizeof(DevView) * (size_t)nv;
  const size_t bytes = vbytes + (sets ? sizeof(ViewSet) * (size_t)nv : 0);
  void *before = pl->p_views.p;
  GS_TRY(ensure(pl, pl->p_views, bytes, s));
  if (pl->p_views.p != before) pl->up_valid = false;
  const bool same_sets =
      sets ? (pl->up_sets.size() == (size_t)nv &&
              std::memcmp(pl->up_sets.data(), sets, sizeof(ViewSet) * (size_t)nv) == 0)
           : pl->up_sets.empty();
  if (pl->up_valid && same_sets && pl->up_views.size() == (size_t)nv &&
      std::memcmp(pl->up_views.data(), views, sizeof(gs_view) * (size_t)nv) == 0)
    return GS_OK;
  const int k = pl->stage_next;
  pl->stage_next = (k + 1) % gs_plan::kStageRing;
  if (pl->stage_pending[k]) {
    if (hipEventSynchronize(pl->stage_done[k]) != hipSuccess)
      return fail(GS_EHIP, "hipEventSynchronize");
    pl->stage_pending[k] = false;
  }
  if (pl->stage_cap[k] < bytes) {
    if (pl->reserved) return fail(GS_EINVAL, "the call exceeds the plan's reservation");
    if (pl->stage[k]) (void)hipHostFree(pl->stage[k]);
    pl->stage[k] = nullptr;
    pl->stage_cap[k] = 0;
    if (hipHostMalloc(&pl->stage[k], bytes, hipHostMallocDefault) != hipSuccess)
      return fail(GS_ENOMEM, "pinned staging allocation failed");
    pl->stage_cap[k] = bytes;
  }
  DevView *dv = reinterpret_cast<DevView *>(pl->stage[k]);
  for (int i = 0; i < nv; ++i) dv[i] = make_dev_view(views[i]);
  if (sets)
    std::memcpy(static_cast<char *>(pl->stage[k]) + vbytes, sets, sizeof(ViewSet) * (size_t)nv);
  pl->up_valid = false;
  if (hipMemcpyAsync(pl->p_views.p, pl->stage[k], bytes, hipMemcpyHostToDevice, s) != hipSuccess)
    return fail(GS_EHIP, "view upload failed");
  if (hipEventRecord(pl->stage_done[k], s) != hipSuccess) return fail(GS_EHIP, "hipEventRecord");
  pl->stage_pending[k] = true;
  pl->up_views.assign(views, views + nv);
  if (sets)
    pl->up_sets.assign(sets, sets + nv);
  else
    pl->up_sets.clear();
  pl->up_valid = true;
  return GS_OK;
}

bool same_proj(const gs_plan *pl, const gs_gaussians *g, const gs_view *views, int32_t nv,
               float cutoff) {
  const ProjKey &k = pl->pkey;
  if (!pl->p_valid || k.mean != g->mean || k.scale != g->scale || k.quat != g->quat ||
      k.dens != g->density || k.n != g->n || k.cutoff != cutoff || (int32_t)k.views.size() != nv ||
      pl->pargs.rectify != pl->rectify)
    return false;
  return std::memcmp(k.views.data(), views, sizeof(gs_view) * (size_t)nv) == 0;
}

bool same_vox(const gs_plan *pl, const gs_gaussians *g, const gs_grid *grid, float cutoff) {
  const VoxKey &k = pl->vkey;
  return pl->v_valid && k.mean == g->mean && k.scale == g->scale && k.quat == g->quat &&
         k.dens == g->density && k.n == g->n && k.cutoff == cutoff &&
         std::memcmp(&k.grid, grid, sizeof(gs_grid)) == 0;
}

// Kernel arguments of a projection of nv views of width x height with at
// most M Gaussians per view and R records in all: tiles, binning chunks,
// render parts and the cutoff constants (no buffers yet).
gs_status proj_args(const gs_plan *pl, int32_t nv, int32_t width, int32_t height, int64_t M,
                    int64_t R, float cutoff, ProjArgs &a) {
  a = ProjArgs{};
  a.M = M;
  a.R = R;
  a.V = nv;
  a.width = width;
  a.height = height;
  a.TX = (a.width + kTile - 1) / kTile;
  a.TY = (a.height + kTile - 1) / kTile;
  a.T = a.TX * a.TY;
  if (a.T > kMaxTilesPerGroup)
    return fail(GS_EUNSUPPORTED, "detector has more than 16384 tiles of 16x16 pixels");
  if (a.M > (int64_t)kEntryIndexMask)
    return fail(GS_EUNSUPPORTED, "projection of more than 2^28-1 Gaussians in one call");
  // binning chunks: 4096 Gaussians, halved while fewer than 512 (view, chunk)
  // workgroups would run (few views); render: parts per tile list so that
  // about 8192 workgroups run (one part when there are that many tiles)
  a.cpt = kChunkPerThread;
  while (a.cpt > 1 && (int64_t)nv * ((a.M + (int64_t)kBlock * a.cpt - 1) / ((int64_t)kBlock * a.cpt)) < 512)
    a.cpt /= 2;
  a.C = (int)((a.M + (int64_t)kBlock * a.cpt - 1) / ((int64_t)kBlock * a.cpt));
  {
    const int64_t tiles = (int64_t)nv * a.T;
    a.parts = tiles >= 8192 ? 1 : (int)std::min<int64_t>(16, (8192 + tiles - 1) / tiles);
  }
  cutoff_consts(cutoff, a.kappa, a.thr, a.qmax);
  a.rectify = pl->rectify;
  a.ovf_host = pl->reserved ? pl->ovf_flag_dev : nullptr;
  if ((int64_t)nv * a.T + 1 > 0x7fffffffLL || (int64_t)nv * a.C + 1 > 0x7fffffffLL)
    return fail(GS_EUNSUPPORTED, "too many views in one call");
  return GS_OK;
}

// The binning of arguments a whose views (and sets) are on the device:
// records, tile histograms and scans, the entry count (read back unless the
// plan is reserved) and the scatter into tile lists and slot offsets.
gs_status proj_bin_launch(gs_plan *pl, ProjArgs &a, hipStream_t s) {
  const int nv = a.V;
  const int64_t VM = a.R, VT = (int64_t)nv * a.T, VC = (int64_t)nv * a.C;
  GS_TRY(ensure(pl, pl->p_rec, sizeof(Rec2) * VM, s));
  GS_TRY(ensure(pl, pl->p_hist, 4 * VC * a.T, s));
  GS_TRY(ensure(pl, pl->p_tile_total, 4 * VT, s));
  GS_TRY(ensure(pl, pl->p_tile_start, 4 * (VT + 1), s));
  GS_TRY(ensure(pl, pl->p_chunk_cnt, 4 * VC, s));
  GS_TRY(ensure(pl, pl->p_chunk_start, 4 * (VC + 1), s));
  GS_TRY(ensure(pl, pl->p_offsets, 4 * (VM + 1), s));  // + the slot total
  GS_TRY(ensure(pl, pl->p_totals, 16, s));
  GS_TRY(ensure_skipped(pl, s));
  a.totals = P<unsigned long long>(pl->p_totals);
  StageTimer t_bin(pl, GS_STAGE_PROJ_BIN, s);
  launch_proj_hist(a, P<Rec2>(pl->p_rec), P<uint32_t>(pl->p_hist), P<uint32_t>(pl->p_chunk_cnt),
                   P<unsigned long long>(pl->skipped), s);
  launch_hist_colscan(nv, a.C, a.T, P<uint32_t>(pl->p_hist), P<uint32_t>(pl->p_tile_total), s);
  if (VT <= 32768 && VC <= 32768) {
    // both scans by one workgroup each, in one launch
    launch_scan2(P<uint32_t>(pl->p_tile_total), P<uint32_t>(pl->p_tile_start), (int)VT,
                 P<uint32_t>(pl->p_chunk_cnt), P<uint32_t>(pl->p_chunk_start), (int)VC,
                 P<unsigned long long>(pl->p_totals), s);
  } else {
    // block-sum scratch of the two multi-block scans: 2 * ceil(n / 4096) + 1 entries each
    const int64_t tmp_t = 2 * ((VT + 4095) / 4096) + 1, tmp_c = 2 * ((VC + 4095) / 4096) + 1;
    GS_TRY(ensure(pl, pl->p_scan_tmp, 4 * (size_t)(tmp_t + tmp_c), s));
    launch_scan_big(P<uint32_t>(pl->p_tile_total), P<uint32_t>(pl->p_tile_start), VT,
                    P<uint32_t>(pl->p_scan_tmp), P<unsigned long long>(pl->p_totals), s);
    launch_scan_big(P<uint32_t>(pl->p_chunk_cnt), P<uint32_t>(pl->p_chunk_start), VC,
                    P<uint32_t>(pl->p_scan_tmp) + tmp_t, P<unsigned long long>(pl->p_totals) + 1, s);
  }
  t_bin.stop();
  GS_TRY(check_launch("projection binning"));
  unsigned long long entries;
  if (pl->reserved) {
    // no readback: the scatter keeps what the reserved list and slots hold
    entries = pl->p_list.cap / 8;
    if (!pl->res.forward_only)
      entries = std::min<unsigned long long>(entries, pl->p_slots.cap >= 16 ? (pl->p_slots.cap - 16) / 24 : 0);
    entries = std::min<unsigned long long>(entries, 0xffffffffull);
  } else {
    if (hipMemcpyAsync(pl->readback, pl->p_totals.p, 16, hipMemcpyDeviceToHost, s) != hipSuccess)
      return fail(GS_EHIP, "entry count readback failed");
    GS_TRY(sync_stream(pl, s));
    entries = pl->readback[0];
    if (entries >= 0xffffffffull || pl->readback[1] >= 0xffffffffull) {
      (void)clear_running_skipped(pl, 0, s);
      return fail(GS_EOVERFLOW, "more than 2^32-1 tile entries: split the views over several calls");
    }
    if (entries != pl->readback[1]) {
      (void)clear_running_skipped(pl, 0, s);
      return fail(GS_EHIP, "internal error: tile and Gaussian entry totals differ");
    }
    gs_status st = ensure(pl, pl->p_list, 8 * (size_t)entries, s);
    if (st != GS_OK) {
      (void)clear_running_skipped(pl, 0, s);
      return st;
    }
  }
  a.cap = (uint32_t)entries;
  StageTimer t_sc(pl, GS_STAGE_PROJ_SCATTER, s);
  launch_proj_scatter(a, P<Rec2>(pl->p_rec), P<uint32_t>(pl->p_hist), P<uint32_t>(pl->p_tile_start),
                      P<uint32_t>(pl->p_chunk_start), P<uint2>(pl->p_list),
                      P<uint32_t>(pl->p_offsets), P<unsigned long long>(pl->skipped),
                      P<unsigned long long>(pl->p_totals), s);
  t_sc.stop();
  GS_TRY(check_launch("projection scatter"));
  pl->p_entries = entries;
  return GS_OK;
}

// Projection + binning: records, tile lists and backward slot offsets.
// models/view_model: NULL for a single-model call on g; else view v renders
// models[view_model[v]] (g is then models[view_model[0]]).
gs_status proj_bin(gs_plan *pl, const gs_gaussians *g, const gs_view *views, int32_t nv,
                   float cutoff, hipStream_t s, const gs_gaussians *models = nullptr,
                   const int32_t *view_model = nullptr) {
  pl->p_valid = false;
  int64_t M = g->n, R = 0;
  std::vector<ViewSet> sets;
  if (models) {
    sets.resize((size_t)nv);
    for (int v = 0; v < nv; ++v) {
      const gs_gaussians &m = models[view_model[v]];
      sets[(size_t)v] = ViewSet{m.mean, m.scale, m.quat, m.density, m.n, R};
      R += m.n;
      M = std::max<int64_t>(M, m.n);
    }
  } else {
    R = (int64_t)nv * M;
  }
  ProjArgs a;
  GS_TRY(proj_args(pl, nv, views[0].width, views[0].height, M, R, cutoff, a));
  a.mean = g->mean; a.scale = g->scale; a.quat = g->quat; a.dens = g->density;
  GS_TRY(upload_views(pl, views, nv, s, models ? sets.data() : nullptr));
  a.views = P<DevView>(pl->p_views);
  a.sets = models ? reinterpret_cast<const ViewSet *>(P<DevView>(pl->p_views) + nv) : nullptr;
  GS_TRY(proj_bin_launch(pl, a, s));
  pl->pargs = a;
  pl->pkey.mean = g->mean; pl->pkey.scale = g->scale; pl->pkey.quat = g->quat;
  pl->pkey.dens = g->density; pl->pkey.n = g->n; pl->pkey.cutoff = cutoff;
  pl->pkey.views.assign(views, views + nv);
  pl->p_valid = models == nullptr;  // a multi-model binning serves no backward
  return GS_OK;
}

gs_status vox_bin(gs_plan *pl, const gs_gaussians *g, const gs_grid *grid, float cutoff,
                  hipStream_t s) {
  pl->v_valid = false;
  VoxArgs a{};
  a.mean = g->mean; a.scale = g->scale; a.quat = g->quat; a.dens = g->density;
  a.M = g->n;
  a.nx = grid->nx; a.ny = grid->ny; a.nz = grid->nz;
  for (int k = 0; k < 3; ++k) {
    a.origin[k] = grid->origin[k];
    a.spacing[k] = grid->spacing[k];
  }
  a.TX = (a.nx + kVTile - 1) / kVTile;
  a.TY = (a.ny + kVTile - 1) / kVTile;
  a.TZ = (a.nz + kVTile - 1) / kVTile;
  const int plane = a.TX * a.TY;
  if (plane > kMaxTilesPerGroup) return fail(GS_EUNSUPPORTED, "grid plane has more than 16384 tiles");
  a.layers = std::max(1, std::min(a.TZ, 4096 / plane));
  a.G = (a.TZ + a.layers - 1) / a.layers;
  a.Tg = plane * a.layers;
  // as for the projection: smaller chunks and several parts per tile list
  // when a small grid (the TV block) would leave most of the chip idle
  a.cpt = kChunkPerThread;
  while (a.cpt > 1 && (int64_t)a.G * ((a.M + (int64_t)kBlock * a.cpt - 1) / ((int64_t)kBlock * a.cpt)) < 512)
    a.cpt /= 2;
  a.C = (int)((a.M + (int64_t)kBlock * a.cpt - 1) / ((int64_t)kBlock * a.cpt));
  {
    const int64_t tiles = (int64_t)a.G * a.Tg;
    a.parts = tiles >= 4096 ? 1 : (int)std::min<int64_t>(16, (4096 + tiles - 1) / tiles);
    a.bparts = tiles >= 1024 ? 1 : (int)std::min<int64_t>(16, (1024 + tiles - 1) / tiles);
  }
  cutoff_consts(cutoff, a.kappa, a.thr, a.qmax);
  a.ovf_host = pl->reserved ? pl->ovf_flag_dev : nullptr;
  const int64_t GT = (int64_t)a.G * a.Tg, GC = (int64_t)a.G * a.C;
  const int64_t nb = (a.M + 4095) / 4096 + 1;
  GS_TRY(ensure(pl, pl->v_rec, sizeof(Rec3) * (size_t)a.M, s));
  GS_TRY(ensure(pl, pl->v_count, 4 * (size_t)a.M, s));
  GS_TRY(ensure(pl, pl->v_offsets, 4 * (size_t)(a.M + 1), s));
  GS_TRY(ensure(pl, pl->v_scan_tmp, 4 * (size_t)(2 * nb + 1), s));
  GS_TRY(ensure(pl, pl->v_hist, 4 * (size_t)(GC * a.Tg), s));
  GS_TRY(ensure(pl, pl->v_tile_total, 4 * (size_t)GT, s));
  GS_TRY(ensure(pl, pl->v_tile_start, 4 * (size_t)(GT + 1), s));
  GS_TRY(ensure(pl, pl->v_totals, 16, s));
  GS_TRY(ensure_skipped(pl, s));
  a.totals = P<unsigned long long>(pl->v_totals);
  StageTimer t_bin(pl, GS_STAGE_VOX_BIN, s);
  launch_vox_records(a, P<Rec3>(pl->v_rec), P<uint32_t>(pl->v_count),
                     P<unsigned long long>(pl->skipped) + 1, s);
  launch_scan_big(P<uint32_t>(pl->v_count), P<uint32_t>(pl->v_offsets), a.M,
                  P<uint32_t>(pl->v_scan_tmp), P<unsigned long long>(pl->v_totals) + 1, s);
  launch_vox_hist(a, P<Rec3>(pl->v_rec), P<uint32_t>(pl->v_hist), s);
  launch_hist_colscan(a.G, a.C, a.Tg, P<uint32_t>(pl->v_hist), P<uint32_t>(pl->v_tile_total), s);
  launch_scan2(P<uint32_t>(pl->v_tile_total), P<uint32_t>(pl->v_tile_start), (int)GT, nullptr,
               nullptr, 0, P<unsigned long long>(pl->v_totals), s);
  t_bin.stop();
  GS_TRY(check_launch("voxel binning"));
  unsigned long long entries;
  if (pl->reserved) {
    entries = pl->v_list.cap / 4;
    if (!pl->res.forward_only) entries = std::min<unsigned long long>(entries, pl->v_slots.cap / 40);
    entries = std::min<unsigned long long>(entries, 0xffffffffull);
  } else {
    if (hipMemcpyAsync(pl->readback, pl->v_totals.p, 16, hipMemcpyDeviceToHost, s) != hipSuccess)
      return fail(GS_EHIP, "entry count readback failed");
    GS_TRY(sync_stream(pl, s));
    entries = pl->readback[0];
    if (entries >= 0xffffffffull || pl->readback[1] >= 0xffffffffull) {
      (void)clear_running_skipped(pl, 1, s);
      return fail(GS_EOVERFLOW, "more than 2^32-1 voxel tile entries");
    }
    if (entries != pl->readback[1]) {
      (void)clear_running_skipped(pl, 1, s);
      return fail(GS_EHIP, "internal error: tile and Gaussian entry totals differ");
    }
    gs_status st = ensure(pl, pl->v_list, 4 * (size_t)entries, s);
    if (st != GS_OK) {
      (void)clear_running_skipped(pl, 1, s);
      return st;
    }
  }
  a.cap = (uint32_t)entries;
  StageTimer t_sc(pl, GS_STAGE_VOX_SCATTER, s);
  launch_vox_scatter(a, P<Rec3>(pl->v_rec), P<uint32_t>(pl->v_hist), P<uint32_t>(pl->v_tile_start),
                     P<uint32_t>(pl->v_list), P<unsigned long long>(pl->skipped),
                     P<unsigned long long>(pl->v_totals), s);
  t_sc.stop();
  GS_TRY(check_launch("voxel scatter"));
  pl->vargs = a;
  pl->v_entries = entries;
  pl->vkey.mean = g->mean; pl->vkey.scale = g->scale; pl->vkey.quat = g->quat;
  pl->vkey.dens = g->density; pl->vkey.n = g->n; pl->vkey.cutoff = cutoff;
  pl->vkey.grid = *grid;
  pl->v_valid = true;
  return GS_OK;
}

gs_status check_loss_image(const float *render, const float *measured, int32_t n_img, int32_t h,
                           int32_t w, float lambda_ssim, const float *loss_out, int *nb) {
  if (!render || !measured || !loss_out) return fail(GS_EINVAL, "NULL array argument");
  if (n_img < 1 || h < 1 || w < 1) return fail(GS_EINVAL, "sizes must be >= 1");
  if (!std::isfinite(lambda_ssim)) return fail(GS_EINVAL, "lambda_ssim not finite");
  const int64_t tiles = (int64_t)n_img * ((h + 31) / 32) * ((w + 31) / 32);
  if (tiles > 0x7fffffffLL) return fail(GS_EUNSUPPORTED, "more than 2^31-1 tiles of 32 x 32");
  if ((int64_t)h * w >= (int64_t)1 << 29) return fail(GS_EUNSUPPORTED, "images of 2^29 pixels or more");
  *nb = loss_image_blocks(n_img, h, w);  // at most the number of 32 x 32 tiles
  return GS_OK;
}

// The SSIM + L1 kernel writes one pair of partial sums per wavefront (the
// same kernel with or without the gradient, so the loss is the same number);
// the finish kernel adds them in a fixed order.
void launch_loss_image(const float *render, const float *measured, int n_img, int h, int w,
                       float lambda_ssim, float *loss_out, float *grad, int nb, float *partials,
                       hipStream_t s) {
  launch_ssim_march(render, measured, n_img, h, w, lambda_ssim, grad, partials, s);
  launch_loss_finish(partials, nb, n_img, h, w, lambda_ssim, loss_out, s);
}

// Static scratch of gs_loss_image_noalloc: the per-tile partial sums, two
// floats per tile.  Each device holds its own copy, whose address is looked
// up once per device (the array's name is not a device address on the host).
constexpr int kNoAllocLossTiles = GS_LOSS_IMAGE_NOALLOC_TILES;
constexpr int kMaxNoAllocDevices = 64;
static __device__ __align__(256) float scratch[2 * kNoAllocLossTiles];
std::mutex g_scratch_mu;
float *g_scratch_ptr[kMaxNoAllocDevices] = {};

gs_status noalloc_scratch(float **out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(GS_EHIP, "hipGetDevice failed");
  if (dev < 0 || dev >= kMaxNoAllocDevices)
    return fail(GS_EUNSUPPORTED, "device index beyond the static buffers' table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(GS_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<float *>(p);
  }
  *out = g_scratch_ptr[dev];
  return GS_OK;
}

// A reserved plan whose device has reported an overflow refuses further
// operator calls until gs_plan_check has reported and cleared it.  The flag
// is read without synchronizing, so a call queued before the device set it
// still runs (its chain kernels write nothing when it overflows itself).
gs_status reserved_overflow(const gs_plan *pl) {
  if (pl->reserved && pl->ovf_flag && *(volatile unsigned int *)pl->ovf_flag)
    return fail(GS_EOVERFLOW, "an earlier call on this plan needed more tile entries than "
                              "reserved; gs_plan_check reports and clears it");
  return GS_OK;
}

struct TempPlan {
  gs_plan *p = nullptr;
  bool owned = false;
  ~TempPlan() {
    if (owned && p) gs_plan_destroy(p);
  }
};

}  // namespace

namespace gsk {
void set_last_error(const char *msg) { g_err = msg; }
}  // namespace gsk

extern "C" {

const char *gs_last_error(void) { return g_err.c_str(); }

gs_status gs_plan_create(gs_alloc_fn alloc, gs_free_fn free_fn, void *ctx, gs_plan **out) {
  if (!out) return fail(GS_EINVAL, "out is NULL");
  *out = nullptr;
  if ((alloc == nullptr) != (free_fn == nullptr))
    return fail(GS_EINVAL, "give both alloc and free, or neither");
  gs_plan *p = new (std::nothrow) gs_plan();
  if (!p) return fail(GS_ENOMEM, "plan allocation failed");
  p->alloc = alloc;
  p->free_fn = free_fn;
  p->ctx = ctx;
  if (hipHostMalloc((void **)&p->readback, 4 * sizeof(unsigned long long), hipHostMallocDefault) !=
      hipSuccess) {
    delete p;
    return fail(GS_EHIP, "pinned readback allocation failed");
  }
  if (hipHostMalloc((void **)&p->ovf_flag, sizeof(unsigned int),
                    hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess ||
      hipHostGetDevicePointer((void **)&p->ovf_flag_dev, p->ovf_flag, 0) != hipSuccess) {
    (void)hipGetLastError();
    if (p->ovf_flag) (void)hipHostFree(p->ovf_flag);
    (void)hipHostFree(p->readback);
    delete p;
    return fail(GS_EHIP, "pinned overflow flag allocation failed");
  }
  *p->ovf_flag = 0u;
  for (int k = 0; k < gs_plan::kStageRing; ++k)
    if (hipEventCreateWithFlags(&p->stage_done[k], hipEventDisableTiming) != hipSuccess) {
      for (int j = 0; j < k; ++j) (void)hipEventDestroy(p->stage_done[j]);
      (void)hipHostFree(p->ovf_flag);
      (void)hipHostFree(p->readback);
      delete p;
      return fail(GS_EHIP, "hipEventCreate failed");
    }
  *out = p;
  return GS_OK;
}

void gs_plan_destroy(gs_plan *p) {
  if (!p) return;
  // wait for the plan's own work only: its last stream and its view uploads
  if (p->used) (void)hipStreamSynchronize(p->last_stream);
  for (int k = 0; k < gs_plan::kStageRing; ++k)
    if (p->stage_pending[k]) (void)hipEventSynchronize(p->stage_done[k]);
  Buf *bufs[] = {&p->p_views, &p->p_rec, &p->p_hist, &p->p_tile_total, &p->p_tile_start,
                 &p->p_chunk_cnt, &p->p_chunk_start, &p->p_offsets, &p->p_list, &p->p_slots,
                 &p->p_totals, &p->p_part, &p->p_scan_tmp, &p->p_fpart, &p->v_rec, &p->v_count, &p->v_offsets, &p->v_scan_tmp, &p->v_hist,
                 &p->v_tile_total, &p->v_tile_start, &p->v_list, &p->v_slots, &p->v_totals,
                 &p->v_fpart,
                 &p->l_coef, &p->l_part, &p->skipped, &p->d_action, &p->d_count, &p->d_offsets,
                 &p->d_scan_tmp, &p->d_totals, &p->m_sse, &p->m_max, &p->m_out, &p->m_stack,
                 &p->m_loss};
  for (Buf *b : bufs) release(p, *b);
  for (int k = 0; k < gs_plan::kStageRing; ++k) {
    if (p->stage[k]) (void)hipHostFree(p->stage[k]);
    if (p->stage_done[k]) (void)hipEventDestroy(p->stage_done[k]);
  }
  if (p->readback) (void)hipHostFree(p->readback);
  if (p->ovf_flag) (void)hipHostFree(p->ovf_flag);
  for (auto &t : p->timed) {
    (void)hipEventDestroy(t.a);
    (void)hipEventDestroy(t.b);
  }
  for (hipEvent_t e : p->event_pool) (void)hipEventDestroy(e);
  delete p;
}

gs_status gs_plan_status(gs_plan *p, int64_t *skipped, int64_t *tile_entries) {
  if (!p) return fail(GS_EINVAL, "plan is NULL");
  if (skipped) *skipped = 0;
  if (tile_entries) *tile_entries = 0;
  if (!p->used || !p->skipped.p) return GS_OK;
  GS_TRY(sync_stream(p, p->last_stream));
  unsigned long long h[8] = {};
  if (hipMemcpy(h, p->skipped.p, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess)
    return fail(GS_EHIP, "status readback failed");
  if (skipped) *skipped = (int64_t)(h[2] + h[3]);
  if (tile_entries) {
    // entries the last binning of each operator needed (a reserved plan
    // keeps at most its reservation, but counts them all)
    int64_t e = 0;
    if (p->reserved) {
      unsigned long long t = 0;
      if (p->p_valid && p->p_totals.p) {
        if (hipMemcpy(&t, p->p_totals.p, 8, hipMemcpyDeviceToHost) != hipSuccess)
          return fail(GS_EHIP, "status readback failed");
        e += (int64_t)t;
      }
      if (p->v_valid && p->v_totals.p) {
        if (hipMemcpy(&t, p->v_totals.p, 8, hipMemcpyDeviceToHost) != hipSuccess)
          return fail(GS_EHIP, "status readback failed");
        e += (int64_t)t;
      }
    } else {
      e = (int64_t)(p->p_valid ? p->p_entries : 0) + (int64_t)(p->v_valid ? p->v_entries : 0);
    }
    *tile_entries = e;
  }
  if (p->reserved && (h[6] || h[7]))
    return fail(GS_EOVERFLOW, std::to_string(h[6] + h[7]) +
                                  " call(s) needed more tile entries than reserved; "
                                  "gs_plan_check reports and clears it");
  return GS_OK;
}

}  // extern "C"

namespace {

gs_status check_reserve(const gs_reserve *r) {
  if (r->max_gaussians < 0 || r->max_gaussians > 0x7fffffffLL || r->max_views < 0 ||
      r->max_proj_entries < 0 || r->max_proj_entries >= 0xffffffffLL || r->max_vox_entries < 0 ||
      r->max_vox_entries >= 0xffffffffLL || r->max_tv_voxels < 0 || r->max_records < 0 ||
      (r->max_views > 0 && (r->width < 1 || r->height < 1 || r->width > 16384 || r->height > 16384)) ||
      (r->nx < 0 || r->ny < 0 || r->nz < 0 || r->nx > 16384 || r->ny > 16384 || r->nz > 16384))
    return fail(GS_EINVAL, "reservation sizes out of range");
  return GS_OK;
}

// The workspace of a reservation: take(buffer, bytes) for every buffer, in
// one place for allocating it and for counting its bytes; with staging, the
// pinned host staging ring for the view constants is sized too.
template <class Take>
gs_status reserve_layout(gs_plan *p, const gs_reserve *r, bool staging, Take take) {
  const int64_t M = std::max<int64_t>(r->max_gaussians, 1);
  const int64_t Cmax16 = (M + 4095) / 4096;  // chunks at the largest chunk size
  if (r->max_views > 0) {
    const int64_t V = r->max_views;
    const int64_t T = (int64_t)((r->width + kTile - 1) / kTile) * ((r->height + kTile - 1) / kTile);
    if (T > kMaxTilesPerGroup) return fail(GS_EUNSUPPORTED, "detector has more than 16384 tiles");
    // binning chunks shrink only while views x chunks < 512, so views x chunks
    // stays below max(V ceil(M / 4096), 1024 + V) for any M' <= M and V' <= V
    const int64_t VC = std::max<int64_t>(V * Cmax16, 1024 + V);
    const int64_t VT = V * T, E = r->max_proj_entries;
    const int64_t R = r->max_records > 0 ? r->max_records : V * M;
    GS_TRY(take(p->p_views, (sizeof(DevView) + sizeof(ViewSet)) * V));
    GS_TRY(take(p->p_rec, sizeof(Rec2) * R));
    GS_TRY(take(p->p_hist, 4 * VC * T));
    GS_TRY(take(p->p_tile_total, 4 * VT));
    GS_TRY(take(p->p_tile_start, 4 * (VT + 1)));
    GS_TRY(take(p->p_chunk_cnt, 4 * VC));
    GS_TRY(take(p->p_chunk_start, 4 * (VC + 1)));
    GS_TRY(take(p->p_offsets, 4 * (R + 1)));
    GS_TRY(take(p->p_totals, 16));
    GS_TRY(take(p->p_scan_tmp, 4 * (size_t)(2 * ((VT + 4095) / 4096) + 2 * ((VC + 4095) / 4096) + 2)));
    GS_TRY(take(p->p_list, 8 * (size_t)std::max<int64_t>(E, 1)));
    if (!r->forward_only) {
      GS_TRY(take(p->p_slots, 24 * (size_t)std::max<int64_t>(E, 1) + 16));
      GS_TRY(take(p->p_part, 72 * (size_t)proj_chain_chunks((int)V) * (size_t)M));
    }
    // render parts x tiles stays below 8192 + tiles
    GS_TRY(take(p->p_fpart, 4 * (size_t)kBlock * (size_t)(8192 + VT)));
    // the loss kernels write at most one pair of partial sums per 32 x 32
    // tile, whichever of them a stack of up to V images takes
    GS_TRY(take(p->l_part, 8 * (size_t)ssim_num_blocks((int)V, r->height, r->width)));
    for (int k = 0; staging && k < gs_plan::kStageRing; ++k) {
      const size_t bytes = (sizeof(DevView) + sizeof(ViewSet)) * (size_t)V;
      if (p->stage_cap[k] < bytes) {
        if (p->stage_pending[k] && hipEventSynchronize(p->stage_done[k]) != hipSuccess)
          return fail(GS_EHIP, "hipEventSynchronize");
        p->stage_pending[k] = false;
        if (p->stage[k]) (void)hipHostFree(p->stage[k]);
        p->stage[k] = nullptr;
        p->stage_cap[k] = 0;
        if (hipHostMalloc(&p->stage[k], bytes, hipHostMallocDefault) != hipSuccess)
          return fail(GS_ENOMEM, "pinned staging allocation failed");
        p->stage_cap[k] = bytes;
      }
    }
  }
  if (r->nx > 0 && r->ny > 0 && r->nz > 0) {
    const int64_t TX = (r->nx + kVTile - 1) / kVTile, TY = (r->ny + kVTile - 1) / kVTile,
                  TZ = (r->nz + kVTile - 1) / kVTile;
    if (TX * TY > kMaxTilesPerGroup) return fail(GS_EUNSUPPORTED, "grid plane has more than 16384 tiles");
    // a group holds max(1, 4096 / plane) tile planes, so tiles per group <=
    // max(4096, plane) and groups x tiles per group <= tiles + that; groups
    // x chunks as for the projection
    const int64_t Tg = std::max<int64_t>(4096, TX * TY), GT = TX * TY * TZ + Tg, G = TZ;
    const int64_t GC = std::max<int64_t>(G * Cmax16, 1024 + G);
    const int64_t E = r->max_vox_entries, nb = (M + 4095) / 4096 + 1;
    GS_TRY(take(p->v_rec, sizeof(Rec3) * (size_t)M));
    GS_TRY(take(p->v_count, 4 * (size_t)M));
    GS_TRY(take(p->v_offsets, 4 * (size_t)(M + 1)));
    GS_TRY(take(p->v_scan_tmp, 4 * (size_t)(2 * nb + 1)));
    GS_TRY(take(p->v_hist, 4 * (size_t)(GC * Tg)));
    GS_TRY(take(p->v_tile_total, 4 * (size_t)GT));
    GS_TRY(take(p->v_tile_start, 4 * (size_t)(GT + 1)));
    GS_TRY(take(p->v_totals, 16));
    GS_TRY(take(p->v_list, 4 * (size_t)std::max<int64_t>(E, 1)));
    if (!r->forward_only) GS_TRY(take(p->v_slots, 40 * (size_t)std::max<int64_t>(E, 1)));
    GS_TRY(take(p->v_fpart, 4 * 2 * (size_t)kBlock * (size_t)(4096 + GT)));  // parts x tiles
  }
  if (r->max_tv_voxels > 0) {
    const size_t nb = (size_t)((r->max_tv_voxels + kBlock - 1) / kBlock);
    GS_TRY(take(p->l_part, 4 * nb));
  }
  return GS_OK;
}

}  // namespace

extern "C" {

gs_status gs_plan_reserve(gs_plan *p, const gs_reserve *r, hipStream_t s) {
  if (!p || !r) return fail(GS_EINVAL, "plan or reservation is NULL");
  GS_TRY(check_reserve(r));
  p->reserved = false;  // allocate first
  p->used = true;
  p->last_stream = s;
  GS_TRY(ensure_skipped(p, s));
  GS_TRY(reserve_layout(p, r, true,
                        [&](Buf &b, size_t bytes) { return ensure(p, b, bytes, s, true); }));
  GS_TRY(sync_stream(p, s));
  p->res = *r;
  p->reserved = true;
  return GS_OK;
}

gs_status gs_plan_reserve_bytes(const gs_reserve *r, int64_t *bytes) {
  if (!r || !bytes) return fail(GS_EINVAL, "reservation or bytes is NULL");
  GS_TRY(check_reserve(r));
  gs_plan tmp;  // holds no memory: only its buffer slots are named
  std::vector<std::pair<const Buf *, size_t>> sizes;
  GS_TRY(reserve_layout(&tmp, r, false, [&](Buf &b, size_t n) {
    n = (std::max<size_t>(n, 256) + 255) & ~(size_t)255;
    for (auto &e : sizes)
      if (e.first == &b) {
        e.second = std::max(e.second, n);
        return GS_OK;
      }
    sizes.emplace_back(&b, n);
    return GS_OK;
  }));
  int64_t total = 64;  // control words
  for (auto &e : sizes) total += (int64_t)e.second;
  *bytes = total;
  return GS_OK;
}

gs_status gs_plan_check(gs_plan *p, int64_t *max_proj_entries, int64_t *max_vox_entries) {
  if (!p) return fail(GS_EINVAL, "plan is NULL");
  if (max_proj_entries) *max_proj_entries = 0;
  if (max_vox_entries) *max_vox_entries = 0;
  if (!p->skipped.p) return GS_OK;
  if (p->used) GS_TRY(sync_stream(p, p->last_stream));
  unsigned long long h[8];
  if (hipMemcpy(h, p->skipped.p, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess)
    return fail(GS_EHIP, "check readback failed");
  if (max_proj_entries) *max_proj_entries = (int64_t)h[4];
  if (max_vox_entries) *max_vox_entries = (int64_t)h[5];
  if (hipMemset(reinterpret_cast<unsigned long long *>(p->skipped.p) + 4, 0, 32) != hipSuccess)
    return fail(GS_EHIP, "check reset failed");
  *(volatile unsigned int *)p->ovf_flag = 0u;
  if (h[6] || h[7])
    return fail(GS_EOVERFLOW, std::to_string(h[6] + h[7]) +
                                  " call(s) needed more tile entries than reserved");
  return GS_OK;
}

gs_status gs_plan_set_rectify(gs_plan *p, int32_t enable) {
  if (!p) return fail(GS_EINVAL, "plan is NULL");
  p->rectify = enable != 0;
  return GS_OK;
}

gs_status gs_project_mean_mu(const gs_gaussians *g, const gs_view *views, int32_t n_views,
                             float *mu_out, float *density_out, gs_plan *plan,
                             hipStream_t stream) {
  GS_TRY(check_gaussians(g));
  GS_TRY(check_views(views, n_views));
  if (!mu_out && !density_out) return fail(GS_EINVAL, "mu_out and density_out are both NULL");
  if (!plan) return fail(GS_EINVAL, "plan is NULL");
  plan->used = true;
  plan->last_stream = stream;
  if (g->n == 0) return GS_OK;
  ProjArgs a{};
  a.mean = g->mean; a.scale = g->scale; a.quat = g->quat; a.dens = g->density;
  a.M = g->n;
  a.V = n_views;
  GS_TRY(upload_views(plan, views, n_views, stream));
  a.views = P<DevView>(plan->p_views);
  plan->p_valid = false;  // the view buffer now holds these views
  launch_mean_mu(a, mu_out, density_out, stream);
  return check_launch("mean rectification factor");
}

gs_status gs_plan_set_timing(gs_plan *p, int32_t enable) {
  if (!p) return fail(GS_EINVAL, "plan is NULL");
  p->timing = enable != 0;
  return GS_OK;
}

gs_status gs_plan_stage_times(gs_plan *p, double *ms_sum, int64_t *count, int32_t n) {
  if (!p) return fail(GS_EINVAL, "plan is NULL");
  if (n < 0 || n > GS_N_STAGES || (n > 0 && (!ms_sum || !count)))
    return fail(GS_EINVAL, "bad output arrays");
  for (int i = 0; i < n; ++i) {
    ms_sum[i] = 0.0;
    count[i] = 0;
  }
  if (p->used && !p->timed.empty()) GS_TRY(sync_stream(p, p->last_stream));
  gs_status st = GS_OK;
  for (auto &t : p->timed) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, t.a, t.b) != hipSuccess)
      st = fail(GS_EHIP, "hipEventElapsedTime failed");
    else if (t.stage < n) {
      ms_sum[t.stage] += ms;
      count[t.stage] += 1;
    }
    p->event_pool.push_back(t.a);
    p->event_pool.push_back(t.b);
  }
  p->timed.clear();
  return st;
}

gs_status gs_view_cone(double theta, float src_obj, float src_det, int32_t width, int32_t height,
                       float pitch, gs_view *out) {
  if (!out) return fail(GS_EINVAL, "out is NULL");
  if (!std::isfinite(theta)) return fail(GS_EINVAL, "theta not finite");
  if (!finite_pos(src_obj) || !std::isfinite(src_det) || !(src_det > src_obj))
    return fail(GS_EINVAL, "need 0 < src_obj < src_det");
  if (width < 1 || height < 1 || width > 16384 || height > 16384)
    return fail(GS_EINVAL, "detector size out of 1..16384");
  if (!finite_pos(pitch)) return fail(GS_EINVAL, "pitch must be > 0");
  const double s = std::sin(theta), c = std::cos(theta);
  const double W[9] = {-s, c, 0.0, 0.0, 0.0, -1.0, -c, -s, 0.0};
  std::memset(out, 0, sizeof(*out));
  out->beam = GS_CONE;
  out->width = width;
  out->height = height;
  out->pitch_u = out->pitch_v = pitch;
  for (int k = 0; k < 9; ++k) out->rot[k] = (float)W[k];
  out->src_obj = src_obj;
  out->src_det = src_det;
  return GS_OK;
}

// The projection kernels' size limits, checked before any plan or device
// memory is touched: 16384 tiles of 16x16 per view, 2^28 - 1 Gaussians per
// model (entries carry the index in 28 bits).
static gs_status check_proj_limits(const gs_gaussians *g, const gs_gaussians *models,
                                   const int32_t *view_model, const gs_view *views,
                                   int32_t n_views) {
  const int64_t T = (int64_t)((views[0].width + kTile - 1) / kTile) *
                    ((views[0].height + kTile - 1) / kTile);
  if (T > kMaxTilesPerGroup)
    return fail(GS_EUNSUPPORTED, "detector has more than 16384 tiles of 16x16 pixels");
  int64_t most = g->n;
  if (models)
    for (int v = 0; v < n_views; ++v) most = std::max<int64_t>(most, models[view_model[v]].n);
  if (most > (int64_t)kEntryIndexMask)
    return fail(GS_EUNSUPPORTED, "projection of more than 2^28-1 Gaussians in one call");
  return GS_OK;
}

static gs_status project_fwd(const gs_gaussians *g, const gs_gaussians *models,
                             const int32_t *view_model, const gs_view *views, int32_t n_views,
                             float cutoff, float *image, gs_plan *plan, hipStream_t stream) {
  GS_TRY(check_views(views, n_views));
  GS_TRY(check_cutoff(cutoff));
  if (!image) return fail(GS_EINVAL, "image is NULL");
  GS_TRY(check_proj_limits(g, models, view_model, views, n_views));
  TempPlan tp;
  if (!plan) {
    GS_TRY(gs_plan_create(nullptr, nullptr, nullptr, &tp.p));
    tp.owned = true;
    plan = tp.p;
  }
  GS_TRY(reserved_overflow(plan));
  plan->used = true;
  plan->last_stream = stream;
  const size_t pix = (size_t)n_views * views[0].width * views[0].height;
  int64_t most = g->n;
  if (models)
    for (int v = 0; v < n_views; ++v) most = std::max<int64_t>(most, models[view_model[v]].n);
  if (most == 0) {
    plan->p_valid = false;
    if (hipMemsetAsync(image, 0, sizeof(float) * pix, stream) != hipSuccess)
      return fail(GS_EHIP, "hipMemsetAsync");
    return tp.owned ? sync_stream(plan, stream) : GS_OK;
  }
  GS_TRY(proj_bin(plan, g, views, n_views, cutoff, stream, models, view_model));
  {
    StageTimer t(plan, GS_STAGE_RENDER_FWD, stream);
    float *partial = nullptr;
    if (plan->pargs.parts > 1) {
      GS_TRY(ensure(plan, plan->p_fpart,
                    4 * (size_t)plan->pargs.parts * (size_t)plan->pargs.V * plan->pargs.T * kBlock,
                    stream));
      partial = P<float>(plan->p_fpart);
    }
    launch_render_fwd(plan->pargs, P<Rec2>(plan->p_rec), P<uint2>(plan->p_list),
                      P<uint32_t>(plan->p_tile_start), image, partial, stream);
  }
  GS_TRY(check_launch("render forward"));
  if (tp.owned) GS_TRY(sync_stream(plan, stream));
  return GS_OK;
}

gs_status gs_project_fwd(const gs_gaussians *g, const gs_view *views, int32_t n_views, float cutoff,
                         float *image, gs_plan *plan, hipStream_t stream) {
  GS_TRY(check_gaussians(g));
  return project_fwd(g, nullptr, nullptr, views, n_views, cutoff, image, plan, stream);
}

gs_status gs_project_fwd_multi(const gs_gaussians *models, int32_t n_models,
                               const int32_t *view_model, const gs_view *views, int32_t n_views,
                               float cutoff, float *image, gs_plan *plan, hipStream_t stream) {
  if (!models || n_models < 1) return fail(GS_EINVAL, "models is NULL or n_models < 1");
  if (!view_model) return fail(GS_EINVAL, "view_model is NULL");
  for (int i = 0; i < n_models; ++i) {
    gs_status st = check_gaussians(&models[i]);
    if (st != GS_OK) return fail(st, std::string(gs_last_error()) + " (model " + std::to_string(i) + ")");
  }
  if (n_views < 1) return fail(GS_EINVAL, "n_views < 1");
  for (int v = 0; v < n_views; ++v)
    if (view_model[v] < 0 || view_model[v] >= n_models)
      return fail(GS_EINVAL, "view_model[" + std::to_string(v) + "] out of range");
  return project_fwd(&models[view_model[0]], models, view_model, views, n_views, cutoff, image,
                     plan, stream);
}

static gs_status project_bwd(const gs_gaussians *g, const gs_view *views, int32_t n_views, float cutoff,
                      const float *grad_image, const gs_grads *grads, int32_t accumulate,
                      const ChainStats &st, gs_plan *plan, hipStream_t stream) {
  GS_TRY(check_gaussians(g));
  GS_TRY(check_views(views, n_views));
  GS_TRY(check_cutoff(cutoff));
  GS_TRY(check_proj_limits(g, nullptr, nullptr, views, n_views));
  if (!grad_image) return fail(GS_EINVAL, "grad_image is NULL");
  if (!grads) return fail(GS_EINVAL, "grads is NULL");
  if (!plan) return fail(GS_EINVAL, "plan is NULL");
  GS_TRY(reserved_overflow(plan));
  plan->used = true;
  plan->last_stream = stream;
  if (g->n == 0) return GS_OK;
  if (!same_proj(plan, g, views, n_views, cutoff))
    GS_TRY(proj_bin(plan, g, views, n_views, cutoff, stream));
  const ProjArgs &a = plan->pargs;
  GS_TRY(ensure(plan, plan->p_slots, 24 * (size_t)plan->p_entries + 16, stream));
  GS_TRY(ensure(plan, plan->p_part, 72 * (size_t)proj_chain_chunks(a.V) * (size_t)a.M, stream));
  {
    StageTimer t(plan, GS_STAGE_RENDER_BWD, stream);
    launch_render_bwd(a, P<Rec2>(plan->p_rec), P<uint2>(plan->p_list),
                      P<uint32_t>(plan->p_tile_start), grad_image, P<float>(plan->p_slots), stream);
  }
  {
    StageTimer t(plan, GS_STAGE_PROJ_CHAIN, stream);
    launch_proj_chain(a, P<uint32_t>(plan->p_offsets),
                      P<float>(plan->p_slots), P<float>(plan->p_part), grads->mean, grads->scale,
                      grads->quat, grads->density, accumulate, st, stream);
  }
  return check_launch("projection backward");
}

gs_status gs_project_bwd(const gs_gaussians *g, const gs_view *views, int32_t n_views, float cutoff,
                         const float *grad_image, const gs_grads *grads, int32_t accumulate,
                         gs_plan *plan, hipStream_t stream) {
  return project_bwd(g, views, n_views, cutoff, grad_image, grads, accumulate,
                     ChainStats{nullptr, nullptr, 0.f}, plan, stream);
}

gs_status gs_project_bwd_stats(const gs_gaussians *g, const gs_view *views, int32_t n_views,
                               float cutoff, const float *grad_image, const gs_grads *grads,
                               int32_t accumulate, const gs_grad_stats *stats, gs_plan *plan,
                               hipStream_t stream) {
  if (!stats || !stats->grad_sum || !stats->visible)
    return fail(GS_EINVAL, "stats and its arrays must not be NULL");
  if (!std::isfinite(stats->scale)) return fail(GS_EINVAL, "stats->scale not finite");
  return project_bwd(g, views, n_views, cutoff, grad_image, grads, accumulate,
                     ChainStats{stats->grad_sum, stats->visible, stats->scale}, plan, stream);
}

gs_status gs_voxelize_fwd(const gs_gaussians *g, const gs_grid *grid, float cutoff, float *volume,
                          gs_plan *plan, hipStream_t stream) {
  GS_TRY(check_gaussians(g));
  GS_TRY(check_grid(grid));
  GS_TRY(check_cutoff(cutoff));
  if (!volume) return fail(GS_EINVAL, "volume is NULL");
  TempPlan tp;
  if (!plan) {
    GS_TRY(gs_plan_create(nullptr, nullptr, nullptr, &tp.p));
    tp.owned = true;
    plan = tp.p;
  }
  GS_TRY(reserved_overflow(plan));
  plan->used = true;
  plan->last_stream = stream;
  const size_t nvox = (size_t)grid->nx * grid->ny * grid->nz;
  if (g->n == 0) {
    plan->v_valid = false;
    if (hipMemsetAsync(volume, 0, sizeof(float) * nvox, stream) != hipSuccess)
      return fail(GS_EHIP, "hipMemsetAsync");
    return tp.owned ? sync_stream(plan, stream) : GS_OK;
  }
  GS_TRY(vox_bin(plan, g, grid, cutoff, stream));
  float *partial = nullptr;
  if (plan->vargs.parts > 1) {
    GS_TRY(ensure(plan, plan->v_fpart,
                  4 * (size_t)plan->vargs.parts * (size_t)plan->vargs.G * plan->vargs.Tg * 2 * kBlock,
                  stream));
    partial = P<float>(plan->v_fpart);
  }
  {
    StageTimer t(plan, GS_STAGE_VOX_FWD, stream);
    launch_vox_fwd(plan->vargs, P<Rec3>(plan->v_rec), P<uint32_t>(plan->v_list),
                   P<uint32_t>(plan->v_tile_start), volume, partial, stream);
  }
  GS_TRY(check_launch("voxelize forward"));
  if (tp.owned) GS_TRY(sync_stream(plan, stream));
  return GS_OK;
}

gs_status gs_voxelize_bwd(const gs_gaussians *g, const gs_grid *grid, float cutoff,
                          const float *grad_volume, const gs_grads *grads, int32_t accumulate,
                          gs_plan *plan, hipStream_t stream) {
  GS_TRY(check_gaussians(g));
  GS_TRY(check_grid(grid));
  GS_TRY(check_cutoff(cutoff));
  if (!grad_volume) return fail(GS_EINVAL, "grad_volume is NULL");
  if (!grads) return fail(GS_EINVAL, "grads is NULL");
  if (!plan) return fail(GS_EINVAL, "plan is NULL");
  GS_TRY(reserved_overflow(plan));
  plan->used = true;
  plan->last_stream = stream;
  if (g->n == 0) return GS_OK;
  if (!same_vox(plan, g, grid, cutoff)) GS_TRY(vox_bin(plan, g, grid, cutoff, stream));
  const VoxArgs &a = plan->vargs;
  GS_TRY(ensure(plan, plan->v_slots, 40 * (size_t)plan->v_entries, stream));
  {
    StageTimer t(plan, GS_STAGE_VOX_BWD, stream);
    launch_vox_bwd(a, P<Rec3>(plan->v_rec), P<uint32_t>(plan->v_list),
                   P<uint32_t>(plan->v_tile_start), P<uint32_t>(plan->v_offsets), grad_volume,
                   P<float>(plan->v_slots), stream);
  }
  {
    StageTimer t(plan, GS_STAGE_VOX_CHAIN, stream);
    launch_vox_chain(a, P<uint32_t>(plan->v_offsets),
                     P<float>(plan->v_slots), grads->mean, grads->scale, grads->quat,
                     grads->density, accumulate, stream);
  }
  return check_launch("voxelize backward");
}

gs_status gs_loss_image(const float *render, const float *measured, int32_t n_img, int32_t h,
                        int32_t w, float lambda_ssim, float *loss_out, float *grad, gs_plan *plan,
                        hipStream_t stream) {
  int nb = 0;
  GS_TRY(check_loss_image(render, measured, n_img, h, w, lambda_ssim, loss_out, &nb));
  if (!plan) return fail(GS_EINVAL, "plan is NULL");
  plan->used = true;
  plan->last_stream = stream;
  GS_TRY(ensure(plan, plan->l_part, 2 * sizeof(float) * (size_t)nb, stream));
  StageTimer t(plan, GS_STAGE_LOSS_IMAGE, stream);
  launch_loss_image(render, measured, n_img, h, w, lambda_ssim, loss_out, grad, nb,
                    P<float>(plan->l_part), stream);
  return check_launch("image loss");
}

gs_status gs_loss_image_noalloc(const float *render, const float *measured, int32_t n_img,
                                int32_t h, int32_t w, float lambda_ssim, float *loss_out,
                                float *grad, hipStream_t stream) {
  int nb = 0;
  GS_TRY(check_loss_image(render, measured, n_img, h, w, lambda_ssim, loss_out, &nb));
  // the limit is stated in tiles of 32 x 32; the kernel writes at most one
  // pair of partial sums per tile
  const int64_t tiles = (int64_t)n_img * ((h + 31) / 32) * ((w + 31) / 32);
  if (tiles > kNoAllocLossTiles)
    return fail(GS_EUNSUPPORTED, "n_img x ceil(h/32) x ceil(w/32) = " + std::to_string(tiles) +
                                     " tiles exceeds the " + std::to_string(kNoAllocLossTiles) +
                                     " of the static buffer");
  if (nb > tiles) return fail(GS_EUNSUPPORTED, "loss partial sums exceed the tile count");
  float *part = nullptr;
  GS_TRY(noalloc_scratch(&part));
  launch_loss_image(render, measured, n_img, h, w, lambda_ssim, loss_out, grad, nb, part, stream);
  return check_launch("image loss");
}

gs_status gs_loss_tv(const float *volume, int32_t nx, int32_t ny, int32_t nz, float weight,
                     float *loss_out, float *grad, int32_t accumulate, gs_plan *plan,
                     hipStream_t stream) {
  if (!volume || !loss_out) return fail(GS_EINVAL, "NULL array argument");
  if (nx < 1 || ny < 1 || nz < 1) return fail(GS_EINVAL, "sizes must be >= 1");
  if (!std::isfinite(weight)) return fail(GS_EINVAL, "weight not finite");
  if (!plan) return fail(GS_EINVAL, "plan is NULL");
  plan->used = true;
  plan->last_stream = stream;
  const int nb = tv_num_blocks(nx, ny, nz);
  GS_TRY(ensure(plan, plan->l_part, sizeof(float) * (size_t)nb, stream));
  int n_part = 0;
  StageTimer t(plan, GS_STAGE_LOSS_TV, stream);
  launch_tv(volume, nx, ny, nz, weight, grad, accumulate, P<float>(plan->l_part), &n_part, stream);
  launch_tv_finish(P<float>(plan->l_part), n_part, loss_out, stream);
  return check_launch("total variation");
}

// ------------------------------------------------------ training loop --

namespace {

ParamPtrs param_ptrs(const gs_params *p) {
  return ParamPtrs{p->mean,   p->log_scale, p->quat,      p->density_raw, p->scale,
                   p->density, p->m_mean,   p->m_scale,   p->m_quat,      p->m_density,
                   p->v_mean, p->v_scale,   p->v_quat,    p->v_density};
}

gs_status check_params(const gs_params *p, bool moments) {
  if (!p) return fail(GS_EINVAL, "params is NULL");
  if (!p->mean || !p->log_scale || !p->quat || !p->density_raw || !p->scale || !p->density)
    return fail(GS_EINVAL, "a parameter array is NULL");
  if (moments && (!p->m_mean || !p->m_scale || !p->m_quat || !p->m_density || !p->v_mean ||
                  !p->v_scale || !p->v_quat || !p->v_density))
    return fail(GS_EINVAL, "an Adam moment array is NULL");
  return GS_OK;
}

double softplus_inv_d(double y) { return y > 30.0 ? y : std::log(std::expm1(y)); }

}  // namespace

gs_status gs_adam_step(const gs_params *p, int64_t n, const gs_grads *grads,
                       const gs_adam_config *cfg, hipStream_t stream) {
  return gsk::adam_step_guarded(p, n, grads, cfg, nullptr, nullptr, stream);
}

}  // extern "C"

namespace gsk {

const unsigned long long *plan_control_words(const gs_plan *p) {
  return p ? reinterpret_cast<const unsigned long long *>(p->skipped.p) : nullptr;
}

const unsigned long long *plan_entries_needed(const gs_plan *p, int voxel) {
  if (!p) return nullptr;
  return reinterpret_cast<const unsigned long long *>(voxel ? p->v_totals.p : p->p_totals.p);
}

int64_t plan_entry_capacity(const gs_plan *p, int voxel) {
  if (!p || !p->reserved) return 0;
  return (int64_t)(voxel ? p->v_list.cap / 4 : p->p_list.cap / 8);
}

DevView dev_view(const gs_view &v) { return make_dev_view(v); }

gs_status project_fwd_device(gs_plan *pl, const DevView *views, const ViewSet *sets, int32_t nv,
                             int32_t width, int32_t height, int64_t M_bound, int64_t R_bound,
                             float cutoff, float *image, hipStream_t s) {
  if (!pl || !pl->reserved) return fail(GS_EINVAL, "a reserved plan is required");
  if (!views || !sets || !image || nv < 1 || M_bound < 1 || R_bound < 1)
    return fail(GS_EINVAL, "invalid device projection arguments");
  GS_TRY(check_cutoff(cutoff));
  if (pl->timing) return fail(GS_EINVAL, "stage timing is not available on this path");
  GS_TRY(reserved_overflow(pl));
  pl->used = true;
  pl->last_stream = s;
  pl->p_valid = false;  // a multi-model binning serves no backward
  ProjArgs a;
  GS_TRY(proj_args(pl, nv, width, height, M_bound, R_bound, cutoff, a));
  // the forward's kernels read each view's Gaussians from its set; the
  // single-model pointers stay null
  a.views = views;
  a.sets = sets;
  GS_TRY(proj_bin_launch(pl, a, s));
  pl->pargs = a;
  float *partial = nullptr;
  if (a.parts > 1) {
    GS_TRY(ensure(pl, pl->p_fpart, 4 * (size_t)a.parts * (size_t)a.V * a.T * kBlock, s));
    partial = P<float>(pl->p_fpart);
  }
  launch_render_fwd(a, P<Rec2>(pl->p_rec), P<uint2>(pl->p_list), P<uint32_t>(pl->p_tile_start),
                    image, partial, s);
  return check_launch("render forward");
}

gs_status adam_step_guarded(const gs_params *p, int64_t n, const gs_grads *grads,
                            const gs_adam_config *cfg, const gs_plan *g0, const gs_plan *g1,
                            hipStream_t stream) {
  GS_TRY(check_params(p, true));
  if (!grads || !cfg) return fail(GS_EINVAL, "grads or cfg is NULL");
  if (n < 0) return fail(GS_EINVAL, "n < 0");
  if (cfg->step < 1) return fail(GS_EINVAL, "step must be >= 1");
  if (n == 0) return GS_OK;
  if (!grads->mean || !grads->scale || !grads->quat || !grads->density)
    return fail(GS_EINVAL, "a gradient array is NULL");
  const float lr[4] = {cfg->lr_mean, cfg->lr_scale, cfg->lr_quat, cfg->lr_density};
  for (float l : lr)
    if (!std::isfinite(l) || l < 0.f) return fail(GS_EINVAL, "learning rates must be finite and >= 0");
  const double b1 = 0.9, b2 = 0.999;
  AdamArgs a{};
  a.raw[0] = p->mean; a.raw[1] = p->log_scale; a.raw[2] = p->quat; a.raw[3] = p->density_raw;
  a.m[0] = p->m_mean; a.m[1] = p->m_scale; a.m[2] = p->m_quat; a.m[3] = p->m_density;
  a.v[0] = p->v_mean; a.v[1] = p->v_scale; a.v[2] = p->v_quat; a.v[3] = p->v_density;
  a.grad[0] = grads->mean; a.grad[1] = grads->scale; a.grad[2] = grads->quat;
  a.grad[3] = grads->density;
  a.scale = p->scale;
  a.density = p->density;
  a.n = n;
  for (int k = 0; k < 4; ++k) a.lr[k] = lr[k];
  a.beta1 = (float)b1;
  a.beta2 = (float)b2;
  a.omb1 = (float)(1.0 - b1);
  a.omb2 = (float)(1.0 - b2);
  a.eps = 1e-15f;
  a.bc1_inv = (float)(1.0 / (1.0 - std::pow(b1, cfg->step)));
  a.bc2_inv = (float)(1.0 / (1.0 - std::pow(b2, cfg->step)));
  a.guard[0] = plan_control_words(g0);
  a.guard[1] = plan_control_words(g1);
  launch_adam(a, stream);
  return check_launch("adam step");
}

}  // namespace gsk

extern "C" {

gs_status gs_random_normals(uint64_t seed, uint64_t counter, int64_t n, float *out,
                            hipStream_t stream) {
  if (n < 0 || (n > 0 && !out)) return fail(GS_EINVAL, "n < 0 or out is NULL");
  if (n > ((int64_t)1 << 34)) return fail(GS_EINVAL, "more than 2^34 draws in one call");
  if (n == 0) return GS_OK;
  launch_random_normals(seed, counter, n, out, stream);
  return check_launch("random normals");
}

gs_status gs_params_activate(const gs_params *p, int64_t n, hipStream_t stream) {
  GS_TRY(check_params(p, false));
  if (n < 0) return fail(GS_EINVAL, "n < 0");
  if (n == 0) return GS_OK;
  launch_activate(p->log_scale, p->density_raw, p->scale, p->density, n, 0, stream);
  return check_launch("activate");
}

gs_status gs_params_from_activated(const gs_params *p, int64_t n, hipStream_t stream) {
  GS_TRY(check_params(p, false));
  if (n < 0) return fail(GS_EINVAL, "n < 0");
  if (n == 0) return GS_OK;
  launch_activate(p->log_scale, p->density_raw, p->scale, p->density, n, 1, stream);
  return check_launch("inverse activation");
}

gs_status gs_densify(const gs_params *src, int64_t n, const gs_grad_stats *stats,
                     const float *normals, const gs_densify_config *cfg, gs_params *dst,
                     int64_t dst_capacity, int32_t *action, int64_t *n_out, gs_plan *plan,
                     hipStream_t stream) {
  GS_TRY(check_params(src, true));
  GS_TRY(check_params(dst, true));
  if (!stats || !stats->grad_sum || !stats->visible) return fail(GS_EINVAL, "stats is incomplete");
  if (!cfg || !n_out || !plan) return fail(GS_EINVAL, "cfg, n_out or plan is NULL");
  if (n < 0 || n > 0x3fffffffLL) return fail(GS_EINVAL, "n out of 0..2^30-1");
  if (dst_capacity < 0) return fail(GS_EINVAL, "dst_capacity < 0");
  if (cfg->densify && !normals) return fail(GS_EINVAL, "normals are needed when densifying");
  if (!(cfg->min_density > 0.f) || !(cfg->clone_max_scale > 0.f) ||
      !std::isfinite(cfg->grad_threshold) || !std::isfinite(cfg->min_density) ||
      !std::isfinite(cfg->clone_max_scale))
    return fail(GS_EINVAL, "min_density and clone_max_scale must be > 0, threshold finite");
  plan->used = true;
  plan->last_stream = stream;
  *n_out = 0;
  if (n == 0) return GS_OK;
  GS_TRY(ensure(plan, plan->d_action, 4 * (size_t)n, stream));
  GS_TRY(ensure(plan, plan->d_count, 4 * (size_t)n, stream));
  GS_TRY(ensure(plan, plan->d_offsets, 4 * ((size_t)n + 1), stream));
  GS_TRY(ensure(plan, plan->d_scan_tmp, 4 * (size_t)(2 * ((n + 4095) / 4096) + 1), stream));
  GS_TRY(ensure(plan, plan->d_totals, 8, stream));
  DensifyArgs a{};
  a.src = param_ptrs(src);
  a.dst = param_ptrs(dst);
  a.n = n;
  a.grad_sum = stats->grad_sum;
  a.visible = stats->visible;
  a.normals = normals;
  a.grad_threshold = cfg->grad_threshold;
  a.t_keep = (float)softplus_inv_d((double)cfg->min_density);
  a.t_half = (float)softplus_inv_d(2.0 * (double)cfg->min_density);
  a.t_scale = (float)std::log((double)cfg->clone_max_scale);
  a.log_split = (float)std::log(1.6);
  a.densify = cfg->densify != 0;
  int32_t *act = action ? action : P<int32_t>(plan->d_action);
  launch_densify_count(a, act, P<uint32_t>(plan->d_count), stream);
  launch_scan_big(P<uint32_t>(plan->d_count), P<uint32_t>(plan->d_offsets), n,
                  P<uint32_t>(plan->d_scan_tmp), P<unsigned long long>(plan->d_totals), stream);
  GS_TRY(check_launch("densify count"));
  if (hipMemcpyAsync(plan->readback, plan->d_totals.p, 8, hipMemcpyDeviceToHost, stream) != hipSuccess)
    return fail(GS_EHIP, "densify readback");
  GS_TRY(sync_stream(plan, stream));
  const int64_t total = (int64_t)plan->readback[0];
  *n_out = total;
  if (total > dst_capacity)
    return fail(GS_EOVERFLOW, "densify needs " + std::to_string(total) + " Gaussians, dst holds " +
                                  std::to_string(dst_capacity));
  launch_densify_write(a, act, P<uint32_t>(plan->d_offsets), stream);
  GS_TRY(check_launch("densify write"));
  return sync_stream(plan, stream);
}

gs_status gs_volume_metrics(const float *volume, const float *gt, int32_t nx, int32_t ny, int32_t nz,
                            double *psnr, double *ssim, gs_plan *plan, hipStream_t stream) {
  if (!volume || !gt || !plan) return fail(GS_EINVAL, "volume, gt or plan is NULL");
  if (nx < 1 || ny < 1 || nz < 1) return fail(GS_EINVAL, "sizes must be >= 1");
  plan->used = true;
  plan->last_stream = stream;
  const int64_t N = (int64_t)nx * ny * nz;
  const int nb = metric_num_blocks(N);
  GS_TRY(ensure(plan, plan->m_sse, 8 * (size_t)nb, stream));
  GS_TRY(ensure(plan, plan->m_max, 4 * (size_t)nb, stream));
  GS_TRY(ensure(plan, plan->m_out, 16, stream));
  GS_TRY(ensure(plan, plan->m_loss, 4 * 9, stream));
  launch_metric_sums(volume, gt, N, P<double>(plan->m_sse), P<float>(plan->m_max),
                     P<double>(plan->m_out), stream);
  if (ssim) {
    GS_TRY(ensure(plan, plan->m_stack, 2 * 4 * (size_t)N, stream));
    GS_TRY(ensure(plan, plan->l_coef, 3 * 4 * (size_t)N, stream));
    float *xs = P<float>(plan->m_stack), *ys = xs + N;
    // (slices, rows, columns) of the stacks normal to x, y, z
    const int dims[3][3] = {{nx, nz, ny}, {ny, nz, nx}, {nz, ny, nx}};
    for (int axis = 0; axis < 3; ++axis) {
      const int n = dims[axis][0], h = dims[axis][1], w = dims[axis][2];
      const int nbs = ssim_num_blocks(n, h, w);
      GS_TRY(ensure(plan, plan->l_part, 2 * sizeof(float) * (size_t)nbs, stream));
      launch_slices(volume, nx, ny, nz, axis, P<double>(plan->m_out), xs, stream);
      launch_slices(gt, nx, ny, nz, axis, P<double>(plan->m_out), ys, stream);
      launch_ssim_coeffs(xs, ys, n, h, w, P<float>(plan->l_coef), P<float>(plan->l_part), stream);
      launch_loss_finish(P<float>(plan->l_part), nbs, n, h, w, 0.f, P<float>(plan->m_loss) + 3 * axis,
                         stream);
    }
  }
  GS_TRY(check_launch("volume metrics"));
  double host_out[2];
  float host_loss[9];
  if (hipMemcpyAsync(host_out, plan->m_out.p, 16, hipMemcpyDeviceToHost, stream) != hipSuccess ||
      (ssim && hipMemcpyAsync(host_loss, plan->m_loss.p, 36, hipMemcpyDeviceToHost, stream) !=
                   hipSuccess))
    return fail(GS_EHIP, "metrics readback");
  GS_TRY(sync_stream(plan, stream));
  if (!(host_out[1] > 0.0)) return fail(GS_EINVAL, "max(gt) must be > 0");
  if (psnr) *psnr = 10.0 * std::log10(host_out[1] * host_out[1] / (host_out[0] / (double)N));
  if (ssim) *ssim = ((double)host_loss[2] + (double)host_loss[5] + (double)host_loss[8]) / 3.0;
  return GS_OK;
}

}  // extern "C"
