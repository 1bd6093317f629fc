// Serving loop: worker threads with their own HIP streams and plans, a FIFO
// of arrived requests, merging of same-model projection requests into one
// launch, and admission against an estimated device-memory budget.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/gs_serve.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Worker {
  hipStream_t stream = nullptr;
  gs_plan *plan = nullptr;
  float *scratch = nullptr;
  size_t scratch_cap = 0;  // floats
  std::vector<gs_view> views;
};

}  // namespace

struct gs_server {
  gs_server_config cfg{};
  std::vector<gs_gaussians> models;
  std::vector<Worker> workers;
  // state of one run
  std::mutex mu;
  std::condition_variable cv;
  std::deque<int64_t> queue;
  bool submit_done = false;
  int64_t inflight_bytes = 0;
  const gs_request *reqs = nullptr;
  gs_request_result *res = nullptr;
  Clock::time_point t0;
};

namespace {

double seconds_since(const Clock::time_point &t0) {
  return std::chrono::duration<double>(Clock::now() - t0).count();
}

// Estimated device memory of one launch: records, slot offsets, tile
// histograms, tile lists (about four 16x16 tiles per Gaussian and view) and
// the image; or the voxel records, lists and volume.
int64_t estimate_bytes(const gs_server *s, const gs_request &r, int64_t views) {
  const int64_t M = s->models[r.model].n;
  if (r.kind == GS_REQ_PROJECT) {
    const int64_t w = r.views[0].width, h = r.views[0].height;
    const int64_t T = ((w + 15) / 16) * ((h + 15) / 16);
    const int64_t C = (M + 4095) / 4096;
    return views * (M * (32 + 4 + 4 * 8) + C * T * 4 + w * h * 4);
  }
  const int64_t nv = (int64_t)r.grid.nx * r.grid.ny * r.grid.nz;
  return M * (64 + 8 + 16 * 4) + nv * 4;
}

bool same_batchable(const gs_request &a, const gs_request &b) {
  return a.kind == GS_REQ_PROJECT && b.kind == GS_REQ_PROJECT && a.model == b.model &&
         a.views[0].width == b.views[0].width && a.views[0].height == b.views[0].height;
}

gs_status ensure_scratch(Worker &w, size_t floats) {
  if (w.scratch_cap >= floats) return GS_OK;
  if (w.scratch) {
    (void)hipStreamSynchronize(w.stream);
    (void)hipFree(w.scratch);
    w.scratch = nullptr;
    w.scratch_cap = 0;
  }
  if (hipMalloc(&w.scratch, floats * sizeof(float)) != hipSuccess) {
    (void)hipGetLastError();
    w.scratch = nullptr;
    return GS_ENOMEM;
  }
  w.scratch_cap = floats;
  return GS_OK;
}

// Runs one batch (all projection requests of one model and detector size, or
// a single volume request) on the worker's stream and waits for it.
gs_status execute(gs_server *s, Worker &w, const std::vector<int64_t> &batch) {
  const gs_request &head = s->reqs[batch[0]];
  const gs_gaussians &g = s->models[head.model];
  if (head.kind == GS_REQ_VOLUME) {
    const gs_grid &grid = head.grid;
    float *out = head.out;
    if (!out) {
      gs_status st = ensure_scratch(w, (size_t)grid.nx * grid.ny * grid.nz);
      if (st != GS_OK) return st;
      out = w.scratch;
    }
    gs_status st = gs_voxelize_fwd(&g, &grid, s->cfg.cutoff, out, w.plan, w.stream);
    if (st != GS_OK) return st;
    return hipStreamSynchronize(w.stream) == hipSuccess ? GS_OK : GS_EHIP;
  }
  w.views.clear();
  for (int64_t i : batch)
    w.views.insert(w.views.end(), s->reqs[i].views, s->reqs[i].views + s->reqs[i].n_views);
  const size_t img = (size_t)head.views[0].width * head.views[0].height;
  float *out = nullptr;
  const bool direct = batch.size() == 1 && head.out != nullptr;
  if (direct) {
    out = head.out;
  } else {
    gs_status st = ensure_scratch(w, img * w.views.size());
    if (st != GS_OK) return st;
    out = w.scratch;
  }
  gs_status st = gs_project_fwd(&g, w.views.data(), (int32_t)w.views.size(), s->cfg.cutoff, out,
                                w.plan, w.stream);
  if (st != GS_OK) return st;
  if (!direct) {
    size_t off = 0;
    for (int64_t i : batch) {
      const gs_request &r = s->reqs[i];
      const size_t n = img * (size_t)r.n_views;
      if (r.out && hipMemcpyAsync(r.out, out + off, n * sizeof(float), hipMemcpyDeviceToDevice,
                                  w.stream) != hipSuccess)
        return GS_EHIP;
      off += n;
    }
  }
  return hipStreamSynchronize(w.stream) == hipSuccess ? GS_OK : GS_EHIP;
}

void worker_loop(gs_server *s, Worker &w, int device) {
  (void)hipSetDevice(device);
  for (;;) {
    std::vector<int64_t> batch;
    int64_t bytes = 0;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      for (;;) {
        if (s->queue.empty()) {
          if (s->submit_done) return;
          s->cv.wait(lk);
          continue;
        }
        const int64_t h = s->queue.front();
        const gs_request &head = s->reqs[h];
        const int64_t hv = head.kind == GS_REQ_PROJECT ? head.n_views : 0;
        const int64_t hb = estimate_bytes(s, head, std::max<int64_t>(hv, 1));
        const int64_t room = s->cfg.hbm_budget_bytes - s->inflight_bytes;
        if (hb > s->cfg.hbm_budget_bytes) {  // can never be admitted
          s->queue.pop_front();
          s->res[h].status = GS_ENOMEM;
          s->res[h].start_s = s->res[h].done_s = seconds_since(s->t0);
          s->res[h].latency_s = s->res[h].done_s - s->reqs[h].arrival_s;
          s->res[h].batch_size = 0;
          s->cv.notify_all();
          continue;
        }
        if (hb > room) {  // wait for work in flight to finish
          s->cv.wait(lk);
          continue;
        }
        batch.push_back(h);
        s->queue.pop_front();
        int64_t views = hv;
        bytes = hb;
        if (s->cfg.batching && head.kind == GS_REQ_PROJECT) {
          for (auto it = s->queue.begin(); it != s->queue.end();) {
            const gs_request &r = s->reqs[*it];
            if (same_batchable(head, r) && views + r.n_views <= s->cfg.max_batch_views) {
              const int64_t nb = estimate_bytes(s, head, views + r.n_views);
              if (nb <= room) {
                views += r.n_views;
                bytes = nb;
                batch.push_back(*it);
                it = s->queue.erase(it);
                continue;
              }
            }
            ++it;
          }
        }
        s->inflight_bytes += bytes;
        break;
      }
    }
    const double t_start = seconds_since(s->t0);
    const gs_status st = execute(s, w, batch);
    const double t_done = seconds_since(s->t0);
    {
      std::lock_guard<std::mutex> lk(s->mu);
      for (int64_t i : batch) {
        gs_request_result &r = s->res[i];
        r.start_s = t_start;
        r.done_s = t_done;
        r.latency_s = t_done - s->reqs[i].arrival_s;
        r.batch_size = (int32_t)batch.size();
        r.status = st;
      }
      s->inflight_bytes -= bytes;
    }
    s->cv.notify_all();
  }
}

}  // namespace

extern "C" {

gs_status gs_server_create(const gs_server_config *cfg, gs_server **out) {
  if (!cfg || !out) return GS_EINVAL;
  *out = nullptr;
  if (cfg->n_workers < 1 || cfg->n_workers > 64 || cfg->max_batch_views < 1 ||
      !(cfg->cutoff > 0.f) || cfg->hbm_budget_bytes <= 0)
    return GS_EINVAL;
  gs_server *s = new (std::nothrow) gs_server();
  if (!s) return GS_ENOMEM;
  s->cfg = *cfg;
  s->workers.resize(cfg->n_workers);
  for (auto &w : s->workers) {
    if (hipStreamCreateWithFlags(&w.stream, hipStreamNonBlocking) != hipSuccess ||
        gs_plan_create(nullptr, nullptr, nullptr, &w.plan) != GS_OK) {
      gs_server_destroy(s);
      return GS_EHIP;
    }
  }
  *out = s;
  return GS_OK;
}

void gs_server_destroy(gs_server *s) {
  if (!s) return;
  for (auto &w : s->workers) {
    if (w.stream) (void)hipStreamSynchronize(w.stream);
    if (w.plan) gs_plan_destroy(w.plan);
    if (w.scratch) (void)hipFree(w.scratch);
    if (w.stream) (void)hipStreamDestroy(w.stream);
  }
  delete s;
}

gs_status gs_server_add_model(gs_server *s, const gs_gaussians *g, int32_t *model_id) {
  if (!s || !g || !model_id) return GS_EINVAL;
  if (g->n < 0 || (g->n > 0 && (!g->mean || !g->scale || !g->quat || !g->density)))
    return GS_EINVAL;
  s->models.push_back(*g);
  *model_id = (int32_t)s->models.size() - 1;
  return GS_OK;
}

gs_status gs_server_run(gs_server *s, const gs_request *reqs, int64_t n, double time_scale,
                        gs_request_result *results, double *wall_s) {
  if (!s || (n > 0 && (!reqs || !results)) || n < 0 || !(time_scale >= 0.0)) return GS_EINVAL;
  for (int64_t i = 0; i < n; ++i) {
    const gs_request &r = reqs[i];
    if (r.model < 0 || r.model >= (int32_t)s->models.size()) return GS_EINVAL;
    if (r.kind == GS_REQ_PROJECT) {
      if (r.n_views < 1 || !r.views) return GS_EINVAL;
      for (int k = 1; k < r.n_views; ++k)
        if (r.views[k].width != r.views[0].width || r.views[k].height != r.views[0].height)
          return GS_EINVAL;
    } else if (r.kind != GS_REQ_VOLUME) {
      return GS_EINVAL;
    }
  }
  int device = 0;
  (void)hipGetDevice(&device);
  std::vector<int64_t> order((size_t)n);
  for (int64_t i = 0; i < n; ++i) order[(size_t)i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int64_t a, int64_t b) { return reqs[a].arrival_s < reqs[b].arrival_s; });
  s->reqs = reqs;
  s->res = results;
  s->queue.clear();
  s->submit_done = false;
  s->inflight_bytes = 0;
  for (int64_t i = 0; i < n; ++i) results[i] = gs_request_result{0.0, 0.0, 0.0, 0, GS_OK};
  s->t0 = Clock::now();
  std::vector<std::thread> threads;
  for (auto &w : s->workers) threads.emplace_back(worker_loop, s, std::ref(w), device);
  for (int64_t i : order) {
    const double at = reqs[i].arrival_s * time_scale;
    const double now = seconds_since(s->t0);
    if (at > now) std::this_thread::sleep_for(std::chrono::duration<double>(at - now));
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->queue.push_back(i);
    }
    s->cv.notify_all();
  }
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->submit_done = true;
  }
  s->cv.notify_all();
  for (auto &t : threads) t.join();
  if (wall_s) *wall_s = seconds_since(s->t0);
  if (time_scale != 1.0)
    for (int64_t i = 0; i < n; ++i) results[i].latency_s = results[i].done_s - reqs[i].arrival_s * time_scale;
  for (int64_t i = 0; i < n; ++i)
    if (results[i].status != GS_OK) return (gs_status)results[i].status;
  return GS_OK;
}

}  // extern "C"
