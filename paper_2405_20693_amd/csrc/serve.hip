// Serving loop for many resident Gaussian models on one GPU: projection
// renders (Eq. 7) and volume queries (Eq. 4).
//
// Continuous batching (batching = 1).  Worker threads, each with its own HIP
// stream, a forward-only reserved plan and kInflight output slots, all sized
// when a run starts from the worker's share of the HBM budget.  A worker
// takes the oldest queued request and, for a projection, every other queued
// projection with the same detector size, of any model, while the batch fits
// its reservation; all their views render in one launch
// (gs_project_fwd_multi).  It enqueues the batch, records an event and goes
// back to the queue without waiting, so up to kInflight batches per worker are
// on the device while newly arrived requests are admitted.  Completions are
// observed by polling the events.  No call allocates device memory and no
// stream is synchronized per batch; the workspace in use never exceeds the
// budget.  A batch whose tile lists overflow the reservation (the entry
// estimate of its requests was short) is detected from the entries the device
// needed and its requests are served again one by one; a request that
// overflows alone fails with GS_ENOMEM.
//
// Graph replay (batching = 2): as continuous batching, but a projection
// batch replays a HIP graph captured, when the run starts, for its shape:
// views (padded to a multiple of 8 above 8, at most the reservation's),
// detector size, and model size class (the launch is sized for the largest model of
// the class).  The batch's request state, its views and the Gaussian set of
// each view (padding views get empty sets), is written to pinned host memory
// of the batch's slot and copied to the worker's device buffer before the
// replay; the graph renders into the worker's image buffer, and the results
// are copied to the requests' outputs after it, all on the worker's stream.
// Volume queries are launched directly.
//
// Per request (batching = 0): the plain path, one request per launch on an
// allocating plan, the stream synchronized after each.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "../../include/gs_serve.h"
#include "internal.h"

namespace {

using Clock = std::chrono::steady_clock;

constexpr int kInflight = 2;

struct Batch {
  std::vector<int64_t> reqs;
  int kind = GS_REQ_PROJECT;
  int slot = 0;
  double t_start = 0.0;
  hipEvent_t done = nullptr;
  int64_t cap = 0;  // the reservation's entries for this kind
};

struct Worker {
  hipStream_t stream = nullptr;
  gs_plan *plan = nullptr;
  // continuous batching: output slots and, per slot, the entries the batch
  // needed (pinned, copied from the device after the batch's binning)
  float *slot_buf[kInflight] = {};
  unsigned long long *need = nullptr;
  hipEvent_t ev[kInflight] = {};
  bool slot_busy[kInflight] = {};
  std::deque<Batch> inflight;
  std::vector<gs_view> views;
  std::vector<int32_t> view_model;
  // graph replay: per slot the batch's DevView[lim.views] then
  // ViewSet[lim.views] in pinned memory, their device copy, the image buffer
  // of the replays, and the executable graph of each batch shape
  // (views, width, height, size class)
  void *vs_host[kInflight] = {};
  void *vs_dev = nullptr;
  float *img_dev = nullptr;
  std::map<std::tuple<int, int, int, int>, hipGraphExec_t> graphs;
  // plain path
  float *scratch = nullptr;
  size_t scratch_cap = 0;  // floats
};

// Limits of one worker's reservation.
struct Limits {
  int32_t views = 0, width = 0, height = 0;
  int64_t m_max = 0;  // the largest model
  int64_t records = 0, proj_entries = 0, vox_entries = 0, voxels = 0, slot_floats = 0;
  int32_t nx = 0, ny = 0, nz = 0;
};

}  // namespace

struct gs_server {
  gs_server_config cfg{};
  std::vector<gs_gaussians> models;
  std::vector<Worker> workers;
  Limits lim;
  int64_t reserved_bytes = 0;
  // tile-list entries per view of (model, width, height), per volume query
  // of (model, nx, ny, nz): measured when a run starts
  std::map<std::tuple<int, int, int>, int64_t> view_entries;
  std::map<std::tuple<int, int, int, int>, int64_t> vol_entries;
  // state of one run
  std::mutex mu;
  std::condition_variable cv;
  std::deque<int64_t> queue;
  std::vector<uint8_t> solo;  // per request: serve alone (after an overflow)
  bool submit_done = false;
  int64_t inflight_bytes = 0;  // plain path admission
  const gs_request *reqs = nullptr;
  gs_request_result *res = nullptr;
  Clock::time_point t0;
};

namespace {

double seconds_since(const Clock::time_point &t0) {
  return std::chrono::duration<double>(Clock::now() - t0).count();
}

gs_status err(gs_status st, const std::string &msg) {
  gsk::set_last_error(msg.c_str());
  return st;
}

// ------------------------------------------------------------ plain path --

// Estimated device memory of one plain launch: records, slot offsets, tile
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

// One request on the worker's stream, waited for.
gs_status execute_plain(gs_server *s, Worker &w, int64_t i) {
  const gs_request &r = s->reqs[i];
  const gs_gaussians &g = s->models[r.model];
  float *out = r.out;
  if (r.kind == GS_REQ_VOLUME) {
    if (!out) {
      gs_status st = ensure_scratch(w, (size_t)r.grid.nx * r.grid.ny * r.grid.nz);
      if (st != GS_OK) return st;
      out = w.scratch;
    }
    gs_status st = gs_voxelize_fwd(&g, &r.grid, s->cfg.cutoff, out, w.plan, w.stream);
    if (st != GS_OK) return st;
  } else {
    if (!out) {
      gs_status st = ensure_scratch(w, (size_t)r.views[0].width * r.views[0].height * r.n_views);
      if (st != GS_OK) return st;
      out = w.scratch;
    }
    gs_status st = gs_project_fwd(&g, r.views, r.n_views, s->cfg.cutoff, out, w.plan, w.stream);
    if (st != GS_OK) return st;
  }
  return hipStreamSynchronize(w.stream) == hipSuccess ? GS_OK : GS_EHIP;
}

void plain_loop(gs_server *s, Worker &w, int device) {
  (void)hipSetDevice(device);
  for (;;) {
    int64_t h = -1, bytes = 0;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      for (;;) {
        if (s->queue.empty()) {
          if (s->submit_done) return;
          s->cv.wait(lk);
          continue;
        }
        const int64_t cand = s->queue.front();
        const gs_request &r = s->reqs[cand];
        const int64_t b = estimate_bytes(s, r, r.kind == GS_REQ_PROJECT ? r.n_views : 1);
        if (b > s->cfg.hbm_budget_bytes) {  // can never be admitted
          s->queue.pop_front();
          gs_request_result &o = s->res[cand];
          o.status = GS_ENOMEM;
          o.start_s = o.done_s = seconds_since(s->t0);
          o.latency_s = o.done_s - r.arrival_s;
          s->cv.notify_all();
          continue;
        }
        if (b > s->cfg.hbm_budget_bytes - s->inflight_bytes) {
          s->cv.wait(lk);
          continue;
        }
        s->queue.pop_front();
        s->inflight_bytes += b;
        h = cand;
        bytes = b;
        break;
      }
    }
    const double t_start = seconds_since(s->t0);
    const gs_status st = execute_plain(s, w, h);
    const double t_done = seconds_since(s->t0);
    {
      std::lock_guard<std::mutex> lk(s->mu);
      gs_request_result &o = s->res[h];
      o.start_s = t_start;
      o.done_s = t_done;
      o.latency_s = t_done - s->reqs[h].arrival_s;
      o.batch_size = 1;
      o.status = st;
      s->inflight_bytes -= bytes;
    }
    s->cv.notify_all();
  }
}

// ------------------------------------------------------- continuous path --

int64_t proj_need(const gs_server *s, const gs_request &r) {
  auto it = s->view_entries.find({r.model, r.views[0].width, r.views[0].height});
  const int64_t per_view = it == s->view_entries.end() ? 0 : it->second;
  return (int64_t)r.n_views * per_view;
}

int64_t vol_need(const gs_server *s, const gs_request &r) {
  auto it = s->vol_entries.find({r.model, r.grid.nx, r.grid.ny, r.grid.nz});
  return it == s->vol_entries.end() ? 0 : it->second;
}

// Whether request r alone fits the workers' reservation.
bool fits_alone(const gs_server *s, const gs_request &r) {
  const Limits &L = s->lim;
  if (r.kind == GS_REQ_VOLUME)
    return r.grid.nx <= L.nx && r.grid.ny <= L.ny && r.grid.nz <= L.nz &&
           vol_need(s, r) <= L.vox_entries &&
           (int64_t)r.grid.nx * r.grid.ny * r.grid.nz <= L.slot_floats;
  const int64_t M = s->models[r.model].n;
  return r.n_views <= L.views && r.views[0].width <= L.width && r.views[0].height <= L.height &&
         (int64_t)r.n_views * M <= L.records && proj_need(s, r) <= L.proj_entries &&
         (int64_t)r.n_views * r.views[0].width * r.views[0].height <= L.slot_floats;
}

void fail_request(gs_server *s, int64_t i, gs_status st) {
  gs_request_result &o = s->res[i];
  o.status = st;
  o.start_s = o.done_s = seconds_since(s->t0);
  o.latency_s = o.done_s - s->reqs[i].arrival_s;
  o.batch_size = 0;
}

// log2 of a model's binning chunks of 4096 Gaussians.
int size_class(int64_t m) {
  int c = 0;
  for (int64_t chunks = (m + 4095) / 4096; chunks > 1; chunks >>= 1) ++c;
  return c;
}

// The largest model of size class c (2^(c+1) - 1 chunks), at most m_max.
int64_t class_bound(int c, int64_t m_max) {
  return std::min<int64_t>(m_max, 4096 * ((int64_t{2} << c) - 1));
}

// Views of a graph for a batch of nv views: nv up to 8, else the next
// multiple of 8, at most the reservation's views.
int32_t graph_views(int32_t nv, int32_t lim_views) {
  const int32_t nb = nv <= 8 ? nv : (nv + 7) / 8 * 8;
  return std::min(nb, lim_views);
}

// Takes the next batch from the queue (lock held): the oldest request and,
// for a projection, later queued projections of the same detector size while
// the views, records, entries and output slot stay within the reservation.
bool take_batch(gs_server *s, Batch &b) {
  while (!s->queue.empty()) {
    const int64_t h = s->queue.front();
    const gs_request &head = s->reqs[h];
    if (!fits_alone(s, head)) {
      s->queue.pop_front();
      fail_request(s, h, GS_ENOMEM);
      continue;
    }
    s->queue.pop_front();
    b.reqs.assign(1, h);
    b.kind = head.kind;
    if (head.kind == GS_REQ_VOLUME || s->solo[(size_t)h]) return true;
    const Limits &L = s->lim;
    // merge models of one size class (their binning chunk counts within a
    // factor of two): a launch bins every view in as many chunks as its
    // largest model needs, so a small model would pay for the largest one
    const int head_class = size_class(s->models[head.model].n);
    int64_t views = head.n_views, recs = (int64_t)head.n_views * s->models[head.model].n;
    int64_t need = proj_need(s, head);
    const int64_t pix = (int64_t)head.views[0].width * head.views[0].height;
    for (auto it = s->queue.begin(); it != s->queue.end();) {
      const gs_request &r = s->reqs[*it];
      if (r.kind == GS_REQ_PROJECT && !s->solo[(size_t)*it] && r.views[0].width == head.views[0].width &&
          r.views[0].height == head.views[0].height && size_class(s->models[r.model].n) == head_class) {
        const int64_t v2 = views + r.n_views, r2 = recs + (int64_t)r.n_views * s->models[r.model].n;
        const int64_t n2 = need + proj_need(s, r);
        if (v2 <= std::min<int64_t>(L.views, s->cfg.max_batch_views) && r2 <= L.records &&
            n2 <= L.proj_entries && v2 * pix <= L.slot_floats) {
          views = v2;
          recs = r2;
          need = n2;
          b.reqs.push_back(*it);
          it = s->queue.erase(it);
          continue;
        }
      }
      ++it;
    }
    return true;
  }
  return false;
}

// Captures the worker's graph for batches of nb views of one detector size
// and size class (the stream must have no capture in progress).
gs_status capture_graph(gs_server *s, Worker &w, int32_t nb, int32_t width, int32_t height, int cls,
                        hipGraphExec_t *exec) {
  const Limits &L = s->lim;
  const gsk::DevView *dv = static_cast<const gsk::DevView *>(w.vs_dev);
  const gsk::ViewSet *ds = reinterpret_cast<const gsk::ViewSet *>(dv + L.views);
  if (hipStreamBeginCapture(w.stream, hipStreamCaptureModeRelaxed) != hipSuccess)
    return err(GS_EHIP, "hipStreamBeginCapture failed");
  gs_status st = gsk::project_fwd_device(w.plan, dv, ds, nb, width, height,
                                         class_bound(cls, L.m_max), L.records, s->cfg.cutoff,
                                         w.img_dev, w.stream);
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(w.stream, &graph);
  if (st != GS_OK || e != hipSuccess || !graph) {
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipGetLastError();
    return st != GS_OK ? st : err(GS_EHIP, "hipStreamEndCapture failed");
  }
  const hipError_t ie = hipGraphInstantiate(exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ie != hipSuccess) {
    (void)hipGetLastError();
    return err(GS_EHIP, "hipGraphInstantiate failed");
  }
  return GS_OK;
}

// A projection batch by graph replay: its views and sets to the device, the
// graph of its shape, its results to the requests' outputs.
gs_status submit_graph(gs_server *s, Worker &w, Batch &b) {
  const Limits &L = s->lim;
  const gs_request &head = s->reqs[b.reqs[0]];
  const int32_t width = head.views[0].width, height = head.views[0].height;
  b.cap = gsk::plan_entry_capacity(w.plan, 0);
  gsk::DevView *hv = static_cast<gsk::DevView *>(w.vs_host[b.slot]);
  gsk::ViewSet *hs = reinterpret_cast<gsk::ViewSet *>(hv + L.views);
  int32_t nv = 0;
  int64_t rb = 0;
  for (int64_t i : b.reqs) {
    const gs_request &r = s->reqs[i];
    const gs_gaussians &m = s->models[r.model];
    for (int32_t k = 0; k < r.n_views; ++k, ++nv) {
      hv[nv] = gsk::dev_view(r.views[k]);
      hs[nv] = gsk::ViewSet{m.mean, m.scale, m.quat, m.density, m.n, rb};
      rb += m.n;
    }
  }
  const int32_t nb = graph_views(nv, L.views);
  for (int32_t v = nv; v < nb; ++v) {
    hv[v] = hv[0];
    hs[v] = gsk::ViewSet{hs[0].mean, hs[0].scale, hs[0].quat, hs[0].dens, 0, rb};
  }
  const size_t bytes = (sizeof(gsk::DevView) + sizeof(gsk::ViewSet)) * (size_t)L.views;
  if (hipMemcpyAsync(w.vs_dev, w.vs_host[b.slot], bytes, hipMemcpyHostToDevice, w.stream) !=
      hipSuccess)
    return GS_EHIP;
  const int cls = size_class(s->models[head.model].n);
  const auto key = std::make_tuple((int)nb, (int)width, (int)height, cls);
  auto it = w.graphs.find(key);
  if (it == w.graphs.end()) {  // a shape the run did not foresee
    hipGraphExec_t exec = nullptr;
    const gs_status st = capture_graph(s, w, nb, width, height, cls, &exec);
    if (st != GS_OK) return st;
    it = w.graphs.emplace(key, exec).first;
  }
  if (hipGraphLaunch(it->second, w.stream) != hipSuccess) return GS_EHIP;
  if (hipMemcpyAsync(&w.need[b.slot], gsk::plan_entries_needed(w.plan, 0), 8,
                     hipMemcpyDeviceToHost, w.stream) != hipSuccess)
    return GS_EHIP;
  const size_t img = (size_t)width * height;
  size_t off = 0;
  for (int64_t i : b.reqs) {
    const gs_request &r = s->reqs[i];
    const size_t n = img * (size_t)r.n_views;
    if (r.out && hipMemcpyAsync(r.out, w.img_dev + off, n * sizeof(float), hipMemcpyDeviceToDevice,
                                w.stream) != hipSuccess)
      return GS_EHIP;
    off += n;
  }
  return hipEventRecord(b.done, w.stream) == hipSuccess ? GS_OK : GS_EHIP;
}

// Enqueues a batch on the worker's stream without waiting for it.
gs_status submit(gs_server *s, Worker &w, Batch &b) {
  if (b.kind == GS_REQ_PROJECT && s->cfg.batching == 2) return submit_graph(s, w, b);
  float *out = w.slot_buf[b.slot];
  const gs_request &head = s->reqs[b.reqs[0]];
  gs_status st;
  if (b.kind == GS_REQ_VOLUME) {
    b.cap = gsk::plan_entry_capacity(w.plan, 1);
    st = gs_voxelize_fwd(&s->models[head.model], &head.grid, s->cfg.cutoff, head.out ? head.out : out,
                         w.plan, w.stream);
    if (st != GS_OK) return st;
    if (hipMemcpyAsync(&w.need[b.slot], gsk::plan_entries_needed(w.plan, 1), 8,
                       hipMemcpyDeviceToHost, w.stream) != hipSuccess)
      return GS_EHIP;
  } else {
    b.cap = gsk::plan_entry_capacity(w.plan, 0);
    w.views.clear();
    w.view_model.clear();
    for (int64_t i : b.reqs) {
      const gs_request &r = s->reqs[i];
      w.views.insert(w.views.end(), r.views, r.views + r.n_views);
      w.view_model.insert(w.view_model.end(), (size_t)r.n_views, r.model);
    }
    const bool direct = b.reqs.size() == 1 && head.out != nullptr;
    st = gs_project_fwd_multi(s->models.data(), (int32_t)s->models.size(), w.view_model.data(),
                              w.views.data(), (int32_t)w.views.size(), s->cfg.cutoff,
                              direct ? head.out : out, w.plan, w.stream);
    if (st != GS_OK) return st;
    if (hipMemcpyAsync(&w.need[b.slot], gsk::plan_entries_needed(w.plan, 0), 8,
                       hipMemcpyDeviceToHost, w.stream) != hipSuccess)
      return GS_EHIP;
    if (!direct) {
      const size_t img = (size_t)head.views[0].width * head.views[0].height;
      size_t off = 0;
      for (int64_t i : b.reqs) {
        const gs_request &r = s->reqs[i];
        const size_t n = img * (size_t)r.n_views;
        if (r.out && hipMemcpyAsync(r.out, out + off, n * sizeof(float), hipMemcpyDeviceToDevice,
                                    w.stream) != hipSuccess)
          return GS_EHIP;
        off += n;
      }
    }
  }
  return hipEventRecord(b.done, w.stream) == hipSuccess ? GS_OK : GS_EHIP;
}

// A completed batch: its requests' results, or (tile lists overflowed) their
// return to the front of the queue to be served one by one.
void finish(gs_server *s, Worker &w, Batch &b, gs_status st) {
  const double t_done = seconds_since(s->t0);
  const bool over = st == GS_OK && (int64_t)w.need[b.slot] > b.cap;
  if (over) {
    int64_t pe = 0, ve = 0;
    (void)gs_plan_check(w.plan, &pe, &ve);  // clears the plan's overflow record
  }
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (over && (b.reqs.size() > 1 || !s->solo[(size_t)b.reqs[0]])) {
      for (auto it = b.reqs.rbegin(); it != b.reqs.rend(); ++it) {
        s->solo[(size_t)*it] = 1;
        s->queue.push_front(*it);
      }
    } else {
      for (int64_t i : b.reqs) {
        gs_request_result &o = s->res[i];
        o.start_s = b.t_start;
        o.done_s = t_done;
        o.latency_s = t_done - s->reqs[i].arrival_s;
        o.batch_size = (int32_t)b.reqs.size();
        o.status = over ? GS_ENOMEM : st;
      }
    }
  }
  w.slot_busy[b.slot] = false;
  s->cv.notify_all();
}

void continuous_loop(gs_server *s, Worker &w, int device) {
  (void)hipSetDevice(device);
  for (;;) {
    // retire the batches that have completed, in order
    while (!w.inflight.empty() && hipEventQuery(w.inflight.front().done) == hipSuccess) {
      finish(s, w, w.inflight.front(), GS_OK);
      w.inflight.pop_front();
    }
    Batch b;
    bool got = false;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      if ((int)w.inflight.size() < kInflight) got = take_batch(s, b);
      if (!got) {
        if (w.inflight.empty()) {
          if (s->submit_done && s->queue.empty()) return;
          s->cv.wait(lk);
          continue;
        }
        if ((int)w.inflight.size() < kInflight) {
          // a slot is free: wait briefly for arrivals, then poll completions
          s->cv.wait_for(lk, std::chrono::microseconds(50));
          continue;
        }
      }
    }
    if (!got) {  // both slots busy: wait for the oldest batch
      (void)hipEventSynchronize(w.inflight.front().done);
      continue;
    }
    int slot = 0;
    while (w.slot_busy[slot]) ++slot;
    w.slot_busy[slot] = true;
    b.slot = slot;
    b.done = w.ev[slot];
    b.t_start = seconds_since(s->t0);
    gs_status st = submit(s, w, b);
    if (st == GS_EOVERFLOW) {
      // an earlier batch on this plan overflowed and the plan refuses calls
      // until it is checked: retire everything in flight, then resubmit
      (void)hipStreamSynchronize(w.stream);
      while (!w.inflight.empty()) {
        finish(s, w, w.inflight.front(), GS_OK);
        w.inflight.pop_front();
      }
      int64_t pe = 0, ve = 0;
      (void)gs_plan_check(w.plan, &pe, &ve);
      st = submit(s, w, b);
    }
    if (st != GS_OK) {
      finish(s, w, b, st);
      continue;
    }
    w.inflight.push_back(b);
  }
}

// Entries per view of every (model, detector) and per volume query of every
// (model, grid shape) in the trace, from one call each on an allocating plan
// (the first request with that key; a volume's entries scaled by 1.5 for
// other offsets, a view's by 1.25 for other angles).
gs_status measure_entries(gs_server *s, const gs_request *reqs, int64_t n, hipStream_t stream) {
  gs_plan *pp = nullptr, *pv = nullptr;
  gs_status st = gs_plan_create(nullptr, nullptr, nullptr, &pp);
  if (st == GS_OK) st = gs_plan_create(nullptr, nullptr, nullptr, &pv);
  if (st != GS_OK) {
    gs_plan_destroy(pp);
    return st;
  }
  float *buf = nullptr;
  size_t cap = 0;
  for (int64_t i = 0; i < n && st == GS_OK; ++i) {
    const gs_request &r = reqs[i];
    const gs_gaussians &g = s->models[r.model];
    size_t need;
    if (r.kind == GS_REQ_PROJECT) {
      if (s->view_entries.count({r.model, r.views[0].width, r.views[0].height})) continue;
      need = (size_t)r.views[0].width * r.views[0].height;
    } else {
      if (s->vol_entries.count({r.model, r.grid.nx, r.grid.ny, r.grid.nz})) continue;
      need = (size_t)r.grid.nx * r.grid.ny * r.grid.nz;
    }
    if (need > cap) {
      if (buf) (void)hipFree(buf);
      buf = nullptr;
      if (hipMalloc(&buf, need * sizeof(float)) != hipSuccess) {
        (void)hipGetLastError();
        st = GS_ENOMEM;
        break;
      }
      cap = need;
    }
    int64_t e = 0;
    if (r.kind == GS_REQ_PROJECT) {
      st = gs_project_fwd(&g, r.views, 1, s->cfg.cutoff, buf, pp, stream);
      if (st == GS_OK) st = gs_plan_status(pp, nullptr, &e);
      s->view_entries[{r.model, r.views[0].width, r.views[0].height}] = e + e / 4 + 256;
    } else {
      st = gs_voxelize_fwd(&g, &r.grid, s->cfg.cutoff, buf, pv, stream);
      if (st == GS_OK) st = gs_plan_status(pv, nullptr, &e);
      s->vol_entries[{r.model, r.grid.nx, r.grid.ny, r.grid.nz}] = e + e / 2 + 4096;
    }
  }
  if (buf) (void)hipFree(buf);
  gs_plan_destroy(pp);
  gs_plan_destroy(pv);
  return st;
}

void release_workers(gs_server *s) {
  for (auto &w : s->workers) {
    if (w.stream) (void)hipStreamSynchronize(w.stream);
    for (auto &b : w.slot_buf) {
      if (b) (void)hipFree(b);
      b = nullptr;
    }
    for (auto &g : w.graphs) (void)hipGraphExecDestroy(g.second);
    w.graphs.clear();
    for (auto &h : w.vs_host) {
      if (h) (void)hipHostFree(h);
      h = nullptr;
    }
    if (w.vs_dev) (void)hipFree(w.vs_dev);
    if (w.img_dev) (void)hipFree(w.img_dev);
    w.vs_dev = nullptr;
    w.img_dev = nullptr;
  }
  s->reserved_bytes = 0;
}

// Graph replay: each worker's request-state buffers and image buffer, and
// its graphs for every batch shape the trace can produce (view counts as
// graph_views pads them, the trace's detector sizes and the size classes of
// its projected models), captured before the run starts.
gs_status prepare_graphs(gs_server *s, const gs_request *reqs, int64_t n) {
  const Limits &L = s->lim;
  if (L.views < 1) return GS_OK;
  std::vector<std::pair<int, int>> sizes;
  std::vector<int> classes;
  for (int64_t i = 0; i < n; ++i) {
    const gs_request &r = reqs[i];
    if (r.kind != GS_REQ_PROJECT) continue;
    const std::pair<int, int> wh(r.views[0].width, r.views[0].height);
    if (std::find(sizes.begin(), sizes.end(), wh) == sizes.end()) sizes.push_back(wh);
    const int c = size_class(s->models[r.model].n);
    if (std::find(classes.begin(), classes.end(), c) == classes.end()) classes.push_back(c);
  }
  std::vector<int32_t> counts;
  for (int32_t nv = 1; nv <= L.views; ++nv) {
    const int32_t nb = graph_views(nv, L.views);
    if (counts.empty() || counts.back() != nb) counts.push_back(nb);
  }
  const size_t vs_bytes = (sizeof(gsk::DevView) + sizeof(gsk::ViewSet)) * (size_t)L.views;
  const size_t img_floats = (size_t)L.views * L.width * L.height;
  for (auto &w : s->workers) {
    if (hipMalloc(&w.vs_dev, vs_bytes) != hipSuccess ||
        hipMalloc(reinterpret_cast<void **>(&w.img_dev), sizeof(float) * img_floats) != hipSuccess) {
      (void)hipGetLastError();
      return err(GS_ENOMEM, "serving graph buffers allocation failed");
    }
    for (auto &h : w.vs_host)
      if (hipHostMalloc(&h, vs_bytes, hipHostMallocDefault) != hipSuccess) {
        h = nullptr;
        return err(GS_ENOMEM, "serving pinned request state allocation failed");
      }
    for (const auto &wh : sizes)
      for (int c : classes)
        for (int32_t nb : counts) {
          const auto key = std::make_tuple((int)nb, wh.first, wh.second, c);
          if (w.graphs.count(key)) continue;
          hipGraphExec_t exec = nullptr;
          const gs_status st = capture_graph(s, w, nb, wh.first, wh.second, c, &exec);
          if (st != GS_OK) return st;
          w.graphs.emplace(key, exec);
        }
  }
  return GS_OK;
}

// Sizes and reserves every worker's plan and output slots for the trace
// within its share of the budget: batches of up to max_batch_views views (at
// least the largest request's) of the largest model at the largest detector,
// and the largest volume query, or, if that does not fit, fewer views per
// batch, then no volume part; requests beyond what fits fail with GS_ENOMEM
// when they are taken.
gs_status reserve_workers(gs_server *s, const gs_request *reqs, int64_t n) {
  Limits base{};
  int64_t m_max = 1, view_need = 0, vol_need_max = 0;
  int32_t req_views = 0;
  for (const auto &g : s->models) m_max = std::max<int64_t>(m_max, g.n);
  for (int64_t i = 0; i < n; ++i) {
    const gs_request &r = reqs[i];
    if (r.kind == GS_REQ_PROJECT) {
      base.width = std::max(base.width, r.views[0].width);
      base.height = std::max(base.height, r.views[0].height);
      req_views = std::max(req_views, r.n_views);
      view_need = std::max(view_need, proj_need(s, r) / std::max(r.n_views, 1));
    } else {
      base.nx = std::max(base.nx, r.grid.nx);
      base.ny = std::max(base.ny, r.grid.ny);
      base.nz = std::max(base.nz, r.grid.nz);
      vol_need_max = std::max(vol_need_max, vol_need(s, r));
    }
  }
  const int64_t share = s->cfg.hbm_budget_bytes / (int64_t)s->workers.size();
  const int32_t v_top = base.width > 0 ? std::max(req_views, s->cfg.max_batch_views) : 0;
  for (int with_vol = base.nx > 0 ? 1 : 0; with_vol >= 0; --with_vol) {
    for (int32_t views = v_top;; views /= 2) {
      Limits L = base;
      if (!with_vol) L.nx = L.ny = L.nz = 0;
      L.voxels = (int64_t)L.nx * L.ny * L.nz;
      L.views = views;
      if (views == 0) L.width = L.height = 0;
      L.records = (int64_t)views * m_max;
      L.m_max = m_max;
      L.proj_entries = std::min<int64_t>((int64_t)views * view_need, 0xfffffffeLL);
      L.vox_entries = with_vol ? std::min<int64_t>(vol_need_max, 0xfffffffeLL) : 0;
      L.slot_floats = std::max<int64_t>((int64_t)views * L.width * L.height, L.voxels);
      gs_reserve r{};
      r.max_gaussians = m_max;
      r.max_views = L.views;
      r.width = L.width;
      r.height = L.height;
      r.max_proj_entries = L.proj_entries;
      r.nx = L.nx;
      r.ny = L.ny;
      r.nz = L.nz;
      r.max_vox_entries = L.vox_entries;
      r.max_records = L.records;
      r.forward_only = 1;
      int64_t bytes = 0;
      gs_status st = gs_plan_reserve_bytes(&r, &bytes);
      if (st != GS_OK) return st;
      bytes += (int64_t)kInflight * L.slot_floats * (int64_t)sizeof(float);
      if (s->cfg.batching == 2)  // the replays' image buffer and request state
        bytes += (int64_t)L.views * L.width * L.height * (int64_t)sizeof(float) +
                 (int64_t)(sizeof(gsk::DevView) + sizeof(gsk::ViewSet)) * L.views;
      if (bytes <= share && (views > 0 || with_vol)) {
        for (auto &w : s->workers) {
          st = gs_plan_reserve(w.plan, &r, w.stream);
          if (st != GS_OK) return st;
          for (auto &b : w.slot_buf)
            if (hipMalloc(&b, sizeof(float) * (size_t)std::max<int64_t>(L.slot_floats, 1)) !=
                hipSuccess) {
              (void)hipGetLastError();
              b = nullptr;
              return err(GS_ENOMEM, "serving output slot allocation failed");
            }
        }
        s->lim = L;
        s->reserved_bytes = bytes * (int64_t)s->workers.size();
        return GS_OK;
      }
      if (views == 0) break;
    }
  }
  s->lim = Limits{};  // nothing fits: every request fails with GS_ENOMEM
  s->reserved_bytes = 0;
  return GS_OK;
}

}  // namespace

extern "C" {

gs_status gs_server_create(const gs_server_config *cfg, gs_server **out) {
  if (!cfg || !out) return GS_EINVAL;
  *out = nullptr;
  if (cfg->n_workers < 1 || cfg->n_workers > 64 || cfg->max_batch_views < 1 ||
      cfg->batching < 0 || cfg->batching > 2 ||
      !(cfg->cutoff > 0.f) || cfg->hbm_budget_bytes <= 0)
    return GS_EINVAL;
  gs_server *s = new (std::nothrow) gs_server();
  if (!s) return GS_ENOMEM;
  s->cfg = *cfg;
  s->workers.resize(cfg->n_workers);
  for (auto &w : s->workers) {
    bool ok = hipStreamCreateWithFlags(&w.stream, hipStreamNonBlocking) == hipSuccess &&
              gs_plan_create(nullptr, nullptr, nullptr, &w.plan) == GS_OK &&
              hipHostMalloc((void **)&w.need, sizeof(unsigned long long) * kInflight,
                            hipHostMallocDefault) == hipSuccess;
    for (auto &e : w.ev) ok = ok && hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess;
    if (!ok) {
      gs_server_destroy(s);
      return GS_EHIP;
    }
  }
  *out = s;
  return GS_OK;
}

void gs_server_destroy(gs_server *s) {
  if (!s) return;
  release_workers(s);
  for (auto &w : s->workers) {
    if (w.plan) gs_plan_destroy(w.plan);
    if (w.scratch) (void)hipFree(w.scratch);
    if (w.need) (void)hipHostFree(w.need);
    for (auto &e : w.ev)
      if (e) (void)hipEventDestroy(e);
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
  const bool cont = s->cfg.batching != 0;
  if (cont) {
    // sizing for this trace (outside the timed run): entries per view and per
    // volume query, then the workers' reservations within the budget
    release_workers(s);
    gs_status st = measure_entries(s, reqs, n, s->workers[0].stream);
    if (st == GS_OK) st = reserve_workers(s, reqs, n);
    if (st == GS_OK && s->cfg.batching == 2) st = prepare_graphs(s, reqs, n);
    if (st != GS_OK) return st;
  }
  std::vector<int64_t> order((size_t)n);
  for (int64_t i = 0; i < n; ++i) order[(size_t)i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int64_t a, int64_t b) { return reqs[a].arrival_s < reqs[b].arrival_s; });
  s->reqs = reqs;
  s->res = results;
  s->queue.clear();
  s->solo.assign((size_t)n, 0);
  s->submit_done = false;
  s->inflight_bytes = 0;
  for (int64_t i = 0; i < n; ++i) results[i] = gs_request_result{0.0, 0.0, 0.0, 0, GS_OK};
  s->t0 = Clock::now();
  std::vector<std::thread> threads;
  for (auto &w : s->workers)
    threads.emplace_back(cont ? continuous_loop : plain_loop, s, std::ref(w), device);
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

gs_status gs_server_reserved_bytes(const gs_server *s, int64_t *bytes) {
  if (!s || !bytes) return GS_EINVAL;
  *bytes = s->reserved_bytes;
  return GS_OK;
}

}  // extern "C"
