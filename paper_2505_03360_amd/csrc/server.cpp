// Serving runtime: continuous batching of collision-evaluation requests from
// several concurrent simulations on one GPU.
//
// Requests arrive from any client thread (bz_serve_submit) with their own
// operator descriptor, distribution buffer, cell list and output buffer.  One
// scheduler thread
//   * admits queued requests as soon as their workspace (ws_per_cell * cells
//     bytes) fits in the caller's arena and an in-flight slot is free, the
//     one with the least estimated work first; a request may be passed by
//     later ones at most kMaxBypass times, after which admission waits for it;
//   * keeps one plan per operator descriptor: the host plan (FP64 tables) is
//     built on a builder thread, so a request that needs a new plan never
//     holds up the admission or completion of the others, and stays cached
//     on the host; its device tables are uploaded into the arena when a
//     request needs them and evicted least-recently-used when idle and
//     memory is short;
//   * launches each admitted request on one of n_streams streams (after the
//     request's ready event, if the caller gave one), so the work of
//     concurrent requests overlaps on the device, and records an event
//     after it;
//   * polls those events, frees the workspace and timestamps completion.
// A request's arithmetic does not depend on the other requests (each has its
// own workspace; per-cell arithmetic is independent of the batch), so its
// result is the same alone and in the mix.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "bz_internal.hpp"

namespace {

constexpr int kMaxBypass = 8;
constexpr size_t kAlign = 256;

uint64_t now_ns() {
  return uint64_t(std::chrono::duration_cast<std::chrono::nanoseconds>(
                      std::chrono::steady_clock::now().time_since_epoch())
                      .count());
}

// First-fit allocator over the caller's arena, 256-byte granules.
struct Arena {
  char* base = nullptr;
  size_t bytes = 0, used = 0, peak = 0;
  std::map<size_t, size_t> free_;  // offset -> size
  void init(void* b, size_t n) {
    base = static_cast<char*>(b);
    bytes = n & ~(kAlign - 1);
    free_.clear();
    if (bytes) free_[0] = bytes;
  }
  bool alloc(size_t sz, size_t* off) {
    sz = bz::align256(std::max<size_t>(sz, 1));
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= sz) {
        *off = it->first;
        const size_t rest = it->second - sz;
        const size_t roff = it->first + sz;
        free_.erase(it);
        if (rest) free_[roff] = rest;
        used += sz;
        peak = std::max(peak, used);
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t sz) {
    sz = bz::align256(std::max<size_t>(sz, 1));
    used -= sz;
    auto it = free_.emplace(off, sz).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
};

// Operator identity of a request: the descriptor without its capacity and
// with an explicit direction table by value.
struct PlanKey {
  bz_plan_desc d{};
  std::vector<double> dirs, weights;
  bz::Strategy sg;  // strategy at the request's size (tune table or heuristics): plans differ by it
  bool operator==(const PlanKey& o) const {
    return sg == o.sg && d.n == o.d.n && d.L == o.d.L && d.R == o.d.R && d.gamma == o.d.gamma &&
           d.kernel_c == o.d.kernel_c && d.m == o.d.m && d.dir_kind == o.d.dir_kind && d.a1 == o.d.a1 &&
           d.a2 == o.d.a2 && d.precision == o.d.precision && d.transform == o.d.transform &&
           d.project == o.d.project && d.chunks == o.d.chunks && d.slices == o.d.slices &&
           d.dealias == o.d.dealias && (d.dim == 2) == (o.d.dim == 2) && dirs == o.dirs &&
           weights == o.weights;
  }
};

PlanKey make_key(const bz_plan_desc& d, int ncells, size_t arena_bytes) {
  PlanKey k;
  k.d = d;
  // a plan picks its strategy from its capacity (tune table or size
  // heuristics; the plain path's stage-A volumes per cell so that the
  // workspace fits a quarter of the arena): requests that resolve to different strategies
  // get (and cache) different plans, built with that strategy as explicit
  // knobs, so a request's arithmetic depends only on its own size
  // (a request's workspace is held to a quarter of the arena, so that several
  // large requests fit at once)
  if (d.dim != 2) k.sg = bz::resolve_strategy(d, std::max(1, ncells), arena_bytes / 4);
  k.d.max_cells = 0;
  k.d.dirs = nullptr;
  k.d.weights = nullptr;
  if (d.dir_kind == BZ_DIRS_EXPLICIT && d.dirs && d.weights && d.m > 0) {
    k.dirs.assign(d.dirs, d.dirs + 3 * size_t(d.m));
    k.weights.assign(d.weights, d.weights + size_t(d.m));
  }
  return k;
}

enum { kPlanBuilding = 0, kPlanReady = 1, kPlanFailed = 2 };

// Host plans built once per operator; device tables present while `resident`.
// Cells per launch: a request larger than this is evaluated in slices, one in
// flight at a time, each on the least loaded stream, so that a long request
// holds a stream for one slice (a few ms) instead of its whole run and shorter
// requests interleave with it; the workspace holds one slice.
int slice_cells(const bz_server_desc& d, const bz_plan_desc& pd) {
  if (d.slice_cells > 0) return d.slice_cells;
  if (pd.dim == 2) return 4096;
  switch (pd.n) {
    case 16: return 2048;
    case 24: return 1024;
    case 32: return 512;
    default: return 256;
  }
}

struct CachedPlan {
  PlanKey key;
  int max_cells = 1;      // capacity the host plan is built for (its strategy follows from it)
  int state = kPlanBuilding;
  bz_status err = BZ_OK;  // build error (kPlanFailed)
  bz_plan* plan = nullptr;
  unsigned char* image = nullptr;  // pinned host copy of the device tables (built with the plan)
  hipEvent_t uploaded = nullptr;   // completion of the last upload of the image into the arena
  bool resident = false;
  size_t tables_off = 0, tables_bytes = 0;
  int inflight = 0;
  uint64_t last_use = 0;
};
// Host plans kept beyond those whose tables are resident.
constexpr size_t kMaxHostPlans = 32;

struct Req {
  uint64_t ticket = 0;
  bz_request r{};
  PlanKey key;
  int state = BZ_REQ_QUEUED;
  bz_status err = BZ_OK;
  uint64_t t_submit = 0, t_admit = 0, t_done = 0;
  int bypassed = 0;
  CachedPlan* cp = nullptr;
  size_t ws_off = 0, ws_bytes = 0;
  hipEvent_t ev = nullptr;
  int slot = -1;  // pinned host word that receives the request's numeric status
  int slice = 0;  // cells per launch (the request is evaluated slice by slice)
  int done_cells = 0;  // cells whose slice has been launched
  int stream = -1;     // stream of the slice in flight (-1: admitted, waiting for its next slice)
  double work = 0.0;   // estimated work of the slice in flight
  int dispatch_bypassed = 0;  // slices of other requests launched while this one waited
};

// Slices queued per stream at most: the server, not the streams' FIFO order,
// decides which request runs next.
constexpr int kStreamDepth = 1;

}  // namespace

struct bz_server {
  bz_server_desc d{};
  Arena arena;
  int device = 0;
  std::vector<hipStream_t> streams;
  std::vector<double> stream_load;  // estimated work of the slices in flight per stream
  std::vector<int> stream_depth;    // slices in flight per stream
  hipStream_t upload = nullptr;
  std::vector<hipEvent_t> event_pool;
  int32_t* status_host = nullptr;  // pinned, one word per in-flight slot
  std::vector<int> free_slots;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<uint64_t> queue;
  std::unordered_map<uint64_t, Req> reqs;
  std::vector<uint64_t> inflight;
  std::vector<std::unique_ptr<CachedPlan>> plans;
  std::deque<CachedPlan*> build_q;  // plans waiting for the builder thread
  std::condition_variable build_cv;
  uint64_t gen = 0;  // bumped by every event the scheduler may wait for (submit, build done, stop)
  uint64_t next_ticket = 1;
  bool stop = false;          // drain and stop the scheduler
  bool builder_stop = false;  // set once the scheduler has drained
  std::thread th, builder;
  // statistics
  std::vector<double> lat_ms;
  uint64_t submitted = 0, completed = 0, failed = 0, cells_done = 0;
  uint64_t t_first_submit = 0, t_last_done = 0;
};

namespace {

void finish(bz_server* s, Req& q, int state, bz_status err) {
  q.state = state;
  q.err = err;
  q.t_done = now_ns();
  if (state == BZ_REQ_DONE) {
    s->completed += 1;
    s->cells_done += uint64_t(q.r.ncells);
    s->lat_ms.push_back(double(q.t_done - q.t_submit) * 1e-6);
    s->t_last_done = q.t_done;
  } else {
    s->failed += 1;
  }
}

hipEvent_t take_event(bz_server* s) {
  if (!s->event_pool.empty()) {
    hipEvent_t e = s->event_pool.back();
    s->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
  return e;
}

// Release a resident plan's table region (after its upload has landed).
void drop_tables(bz_server* s, CachedPlan* c) {
  if (c->uploaded) (void)hipEventSynchronize(c->uploaded);
  s->arena.release(c->tables_off, c->tables_bytes);
  c->resident = false;
}

void free_plan(CachedPlan* c) {
  if (c->uploaded) (void)hipEventSynchronize(c->uploaded);
  if (c->plan) bz_plan_destroy(c->plan);
  if (c->image) (void)hipHostFree(c->image);
  if (c->uploaded) (void)hipEventDestroy(c->uploaded);
  c->plan = nullptr;
  c->image = nullptr;
  c->uploaded = nullptr;
}

// Drop the device tables of idle resident plans (least recently used first)
// until `need` bytes can be allocated or nothing idle is left; their host
// plans stay cached.
bool alloc_with_eviction(bz_server* s, size_t need, size_t* off) {
  while (!s->arena.alloc(need, off)) {
    CachedPlan* victim = nullptr;
    for (auto& c : s->plans)
      if (c->resident && c->inflight == 0 && (!victim || c->last_use < victim->last_use)) victim = c.get();
    if (!victim) return false;
    drop_tables(s, victim);
  }
  return true;
}

// Destroy the least recently used idle host plans beyond kMaxHostPlans.
void trim_host_plans(bz_server* s) {
  while (s->plans.size() > kMaxHostPlans) {
    size_t vi = s->plans.size();
    for (size_t i = 0; i < s->plans.size(); ++i) {
      const CachedPlan* c = s->plans[i].get();
      if (c->state == kPlanBuilding || c->resident || c->inflight) continue;
      if (vi == s->plans.size() || c->last_use < s->plans[vi]->last_use) vi = i;
    }
    if (vi == s->plans.size()) return;
    bool queued = false;  // requests still name it: keep it
    for (uint64_t id : s->queue) queued |= s->reqs[id].cp == s->plans[vi].get();
    if (queued) return;
    free_plan(s->plans[vi].get());
    s->plans.erase(s->plans.begin() + long(vi));
  }
}

// The cached plan of a request's operator; a new one is handed to the
// builder thread and comes back kPlanBuilding.
CachedPlan* find_plan(bz_server* s, Req& q) {
  for (auto& c : s->plans)
    if (c->key == q.key) return c.get();
  auto c = std::make_unique<CachedPlan>();
  c->key = q.key;
  c->max_cells = std::max(1, std::min(q.r.ncells, q.slice));
  s->plans.push_back(std::move(c));
  CachedPlan* cp = s->plans.back().get();
  s->build_q.push_back(cp);
  s->build_cv.notify_one();
  return cp;
}

// Builder thread: FP64 tables of new plans on the host, outside the lock.
void builder(bz_server* s) {
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    s->build_cv.wait(lk, [s] { return s->builder_stop || !s->build_q.empty(); });
    if (s->build_q.empty()) return;  // the scheduler has drained: nothing left to build
    CachedPlan* cp = s->build_q.front();
    s->build_q.pop_front();
    bz_plan_desc d = cp->key.d;
    d.max_cells = cp->max_cells;
    if (d.dim != 2 && !d.dealias) {  // the strategy of the key, as explicit knobs
      d.transform = cp->key.sg.transform;
      d.chunks = cp->key.sg.transform != BZ_XF_FUSED ? cp->key.sg.plain_k : cp->key.sg.chunks;
      d.slices = cp->key.sg.transform != BZ_XF_FUSED ? 0 : cp->key.sg.slices;
    }
    if (d.dir_kind == BZ_DIRS_EXPLICIT) {
      d.dirs = cp->key.dirs.data();
      d.weights = cp->key.weights.data();
    }
    lk.unlock();
    bz_plan* p = nullptr;
    bz_status st = bz_plan_create(&d, &p);
    unsigned char* image = nullptr;
    hipEvent_t ev = nullptr;
    if (st == BZ_OK) {
      // the device image of the tables, pinned so that uploads are asynchronous copies
      if (hipHostMalloc(reinterpret_cast<void**>(&image), p->tables_bytes, hipHostMallocDefault) != hipSuccess ||
          hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
        st = bz::fail(BZ_ERR_DEVICE, "server: pinned table image");
      } else {
        bz::fill_tables_host(p, image);
      }
    }
    lk.lock();
    cp->plan = p;
    cp->image = image;
    cp->uploaded = ev;
    cp->err = st;
    cp->state = st == BZ_OK ? kPlanReady : kPlanFailed;
    if (st == BZ_OK) cp->tables_bytes = p->tables_bytes;
    s->gen += 1;
    s->cv.notify_all();
  }
}

// Upload the tables of a ready plan into the arena (called with the lock
// held; the copy is short).  False if no room is left.
bool make_resident(bz_server* s, CachedPlan* cp, bz_status* err) {
  if (cp->resident) return true;
  if (!alloc_with_eviction(s, cp->tables_bytes, &cp->tables_off)) return false;
  // asynchronous copy from the pinned image; the request's kernels wait for the event
  if (hipMemcpyAsync(s->arena.base + cp->tables_off, cp->image, cp->tables_bytes, hipMemcpyHostToDevice,
                     s->upload) != hipSuccess ||
      hipEventRecord(cp->uploaded, s->upload) != hipSuccess) {
    (void)hipStreamSynchronize(s->upload);
    s->arena.release(cp->tables_off, cp->tables_bytes);
    *err = BZ_ERR_DEVICE;
    return false;
  }
  cp->resident = true;
  return true;
}

// Launch the request's next slice on the least loaded stream (the first one
// after its ready event, with its status word cleared); the status word goes
// to the request's pinned host slot after the last slice.
bz_status launch_slice(bz_server* s, Req& q, int st_i) {
  hipStream_t st = s->streams[size_t(st_i)];
  const bz_plan* p = q.cp->plan;
  const bz::Binding b = bz::make_binding(p, s->arena.base + q.cp->tables_off, s->arena.base + q.ws_off, q.ws_bytes);
  const bool first = q.done_cells == 0;
  if (first && q.r.ready_event && hipStreamWaitEvent(st, static_cast<hipEvent_t>(q.r.ready_event), 0) != hipSuccess)
    return BZ_ERR_DEVICE;
  if (first && hipStreamWaitEvent(st, q.cp->uploaded, 0) != hipSuccess) return BZ_ERR_DEVICE;  // the tables
  if (first) bz::launch_clear_status(b.ws, b.lay, st);
  const int cnt = std::min(q.slice, q.r.ncells - q.done_cells);
  if (cnt > 0) {
    const size_t npts = p->npts;
    const char* f = static_cast<const char*>(q.r.f);
    const int32_t* idx = q.r.idx;
    if (idx) idx += q.done_cells;
    else f += size_t(q.done_cells) * npts * (q.r.f_dtype == BZ_FP32 ? 4 : 8);
    char* out = static_cast<char*>(q.r.q);
    const bool scatter = (q.r.flags & BZ_SCATTER) != 0;
    if (!scatter) out += size_t(q.done_cells) * npts * ((p->project || !p->fp32) ? 8 : 4);
    const bz_status lst = bz::launch_collide(p, b, f, q.r.f_dtype == BZ_FP32, idx, cnt, nullptr, out, scatter, st, false);
    if (lst != BZ_OK) return lst;
  }
  q.done_cells += cnt;
  if (q.done_cells >= q.r.ncells &&
      hipMemcpyAsync(&s->status_host[q.slot], static_cast<char*>(b.ws) + b.lay.status_off, sizeof(int32_t),
                     hipMemcpyDeviceToHost, st) != hipSuccess)
    return BZ_ERR_DEVICE;
  if (hipEventRecord(q.ev, st) != hipSuccess) return BZ_ERR_DEVICE;
  q.stream = st_i;
  q.work = double(std::max(cnt, 1)) * double(p->npts) * double(p->m1);  // cells x grid points x passes
  s->stream_load[size_t(st_i)] += q.work;
  s->stream_depth[size_t(st_i)] += 1;
  return BZ_OK;
}

// Estimated work left of an admitted request (cells x grid points x passes).
double remaining_work(const Req& q) {
  return double(std::max(q.r.ncells - q.done_cells, 1)) * double(q.cp->plan->npts) * double(q.cp->plan->m1);
}

// End an admitted request: free its workspace, slot and event.
void retire(bz_server* s, size_t i, int state, bz_status err) {
  Req& q = s->reqs[s->inflight[i]];
  s->arena.release(q.ws_off, q.ws_bytes);
  q.cp->inflight -= 1;
  if (q.ev) s->event_pool.push_back(q.ev);
  q.ev = nullptr;
  if (q.slot >= 0) s->free_slots.push_back(q.slot);
  q.slot = -1;
  finish(s, q, state, err);
  s->inflight[i] = s->inflight.back();
  s->inflight.pop_back();
  s->gen += 1;
}

// Slices of at most this much work (cells x grid points x passes; a full
// 512-cell slice at n = 32 with 33 passes, about a millisecond of device time,
// is below it, a 256-cell slice at n = 48 above) are short: with two or more
// streams, stream 0 takes only short slices, so a short request never waits
// behind long ones.
constexpr double kShortWork = double(3u << 28);

double next_slice_work(const Req& q) {
  const int cnt = std::max(1, std::min(q.slice, q.r.ncells - q.done_cells));
  return double(cnt) * double(q.cp->plan->npts) * double(q.cp->plan->m1);
}

// Launch slices while a stream has room (fewer than kStreamDepth queued): of
// the waiting requests that can launch now, the one with the least work left
// goes first, on the stream with the fewest (then the lightest) slices queued,
// so short requests overtake long ones at slice boundaries; long slices keep
// off stream 0.  A request passed over by more than kMaxDispatchBypass
// launches goes first (the one passed over most), which bounds how long a long
// request can be held back.
constexpr int kMaxDispatchBypass = 32;

void dispatch(bz_server* s) {
  const bool split = s->streams.size() > 1;
  auto free_stream = [s](int lo) {
    int st_i = -1;
    for (int i = lo; i < int(s->streams.size()); ++i) {
      const size_t a = size_t(i);
      if (s->stream_depth[a] >= kStreamDepth) continue;
      if (st_i < 0) {
        st_i = i;
        continue;
      }
      const size_t b = size_t(st_i);
      if (s->stream_depth[a] < s->stream_depth[b] ||
          (s->stream_depth[a] == s->stream_depth[b] && s->stream_load[a] < s->stream_load[b]))
        st_i = i;
    }
    return st_i;
  };
  for (;;) {
    const int any = free_stream(0);
    if (any < 0) return;
    const int any_long = split ? free_stream(1) : any;
    size_t best = s->inflight.size();
    double best_key = 0.0;
    bool best_urgent = false, best_long = false;
    for (size_t i = 0; i < s->inflight.size(); ++i) {
      const Req& q = s->reqs[s->inflight[i]];
      if (q.stream >= 0) continue;
      const bool lng = split && next_slice_work(q) > kShortWork;
      if (lng && any_long < 0) continue;  // only stream 0 is free
      const bool urgent = q.dispatch_bypassed > kMaxDispatchBypass;
      const double key = urgent ? -double(q.dispatch_bypassed) : remaining_work(q);
      if (best == s->inflight.size() || (urgent && !best_urgent) || (urgent == best_urgent && key < best_key)) {
        best = i;
        best_key = key;
        best_urgent = urgent;
        best_long = lng;
      }
    }
    if (best == s->inflight.size()) return;
    const int st_i = best_long ? any_long : any;
    const uint64_t id = s->inflight[best];
    for (uint64_t o : s->inflight)
      if (o != id && s->reqs[o].stream < 0) s->reqs[o].dispatch_bypassed += 1;
    Req& q = s->reqs[id];
    q.dispatch_bypassed = 0;
    const bz_status lst = launch_slice(s, q, st_i);
    if (lst != BZ_OK) {
      for (auto x : s->streams) (void)hipStreamSynchronize(x);  // nothing of a failed launch stays in flight
      if (q.stream >= 0) {
        s->stream_load[size_t(q.stream)] -= q.work;
        s->stream_depth[size_t(q.stream)] -= 1;
      }
      retire(s, best, BZ_REQ_FAILED, lst);
    }
  }
}

void reap(bz_server* s) {
  for (size_t i = 0; i < s->inflight.size();) {
    Req& q = s->reqs[s->inflight[i]];
    if (q.stream < 0) {  // waiting for its next slice
      ++i;
      continue;
    }
    const hipError_t e = hipEventQuery(q.ev);
    if (e == hipErrorNotReady) {
      ++i;
      continue;
    }
    s->stream_load[size_t(q.stream)] -= q.work;
    s->stream_depth[size_t(q.stream)] -= 1;
    q.stream = -1;
    if (e == hipSuccess && q.done_cells < q.r.ncells) {  // the next slice waits for dispatch
      ++i;
      continue;
    }
    const bool nonfinite = q.slot >= 0 && s->status_host[q.slot] != 0;
    if (e != hipSuccess) retire(s, i, BZ_REQ_FAILED, BZ_ERR_DEVICE);
    else if (nonfinite) retire(s, i, BZ_REQ_FAILED, BZ_ERR_NUMERIC);
    else retire(s, i, BZ_REQ_DONE, BZ_OK);
  }
}

// Workspace and, when needed, tables of request q.  With nothing in flight
// every other plan is idle and evictable, so the only thing that can split
// the free space is this plan's own tables: they are then dropped and placed
// after the workspace (the descriptor check guarantees that both fit).
bool place(bz_server* s, CachedPlan* cp, size_t ws, size_t* off, bz_status* err) {
  cp->inflight += 1;  // pin the plan while allocating
  bool ok = make_resident(s, cp, err) && alloc_with_eviction(s, ws, off);
  if (!ok && *err == BZ_OK && s->inflight.empty()) {
    if (cp->resident) drop_tables(s, cp);
    ok = alloc_with_eviction(s, ws, off);
    if (ok && !make_resident(s, cp, err)) {
      s->arena.release(*off, ws);
      ok = false;
    }
  }
  cp->inflight -= 1;
  return ok;
}

// Queued requests considered per admission round (the oldest ones).
constexpr size_t kAdmitWindow = 256;

// Admits what fits.  Order: requests already passed over more than kMaxBypass
// times first (oldest first), then the others by estimated work (cells x grid
// points x passes, oldest first among equals), so that a short request does
// not wait for a free slot behind long ones.  A request whose workspace
// exceeds a sixteenth of the arena is admitted out of that turn only if an
// eighth of the arena stays free.  Every admission counts as a bypass of each
// older request still queued, which bounds how long a long request can be
// overtaken; once one is past the bound and does not fit, nothing else is
// admitted until it does.  Returns true if any request changed state.
bool admit(bz_server* s) {
  if (int(s->inflight.size()) >= s->d.max_inflight) return false;
  bool progress = false;
  struct Cand {
    size_t pos;
    bool urgent;
    double work;
  };
  std::vector<Cand> cand;
  const size_t window = std::min(s->queue.size(), kAdmitWindow);
  std::vector<char> gone(window, 0);  // admitted or failed in this round
  for (size_t qi = 0; qi < window; ++qi) {
    Req& q = s->reqs[s->queue[qi]];
    CachedPlan* cp = q.cp ? q.cp : find_plan(s, q);
    q.cp = cp;
    if (cp->state == kPlanBuilding) continue;  // waits for the builder, passed by the others
    if (cp->state == kPlanFailed) {
      finish(s, q, BZ_REQ_FAILED, cp->err);
      gone[qi] = 1;
      progress = true;
      continue;
    }
    const double work = double(std::max(q.r.ncells, 1)) * double(cp->plan->npts) * double(cp->plan->m1);
    cand.push_back({qi, q.bypassed > kMaxBypass, work});
  }
  std::stable_sort(cand.begin(), cand.end(), [](const Cand& a, const Cand& b) {
    if (a.urgent != b.urgent) return a.urgent;
    if (a.urgent) return a.pos < b.pos;
    return a.work < b.work;
  });
  std::vector<size_t> admitted;
  for (const Cand& c : cand) {
    if (int(s->inflight.size()) >= s->d.max_inflight) break;
    const uint64_t id = s->queue[c.pos];
    Req& q = s->reqs[id];
    CachedPlan* cp = q.cp;
    const bz_plan* p = cp->plan;
    const size_t ws = p->ws_fixed + p->ws_per_cell * size_t(std::max(1, std::min(q.r.ncells, q.slice)));
    if (bz::align256(ws) + bz::align256(cp->tables_bytes) > s->arena.bytes) {  // can never fit
      finish(s, q, BZ_REQ_FAILED, BZ_ERR_NOMEM);
      gone[c.pos] = 1;
      progress = true;
      continue;
    }
    // headroom: a large workspace is not admitted ahead of its turn if it would
    // leave less than an eighth of the arena free, so that short requests
    // still find room while large ones run
    if (!c.urgent && !s->inflight.empty() && bz::align256(ws) > s->arena.bytes / 16) {
      const size_t need = bz::align256(ws) + (cp->resident ? 0 : bz::align256(cp->tables_bytes));
      if (s->arena.used + need + s->arena.bytes / 8 > s->arena.bytes) continue;
    }
    size_t off = 0;
    bz_status perr = BZ_OK;
    if (!place(s, cp, ws, &off, &perr)) {
      if (perr != BZ_OK) {  // device error while uploading the tables
        finish(s, q, BZ_REQ_FAILED, perr);
        gone[c.pos] = 1;
        progress = true;
        continue;
      }
      if (c.urgent) break;  // no room while others run: the space that frees goes to it
      continue;
    }
    hipEvent_t ev = take_event(s);
    gone[c.pos] = 1;
    progress = true;
    if (!ev) {
      s->arena.release(off, ws);
      finish(s, q, BZ_REQ_FAILED, BZ_ERR_DEVICE);
      continue;
    }
    const int slot = s->free_slots.back();  // at most max_inflight requests are in flight
    s->free_slots.pop_back();
    s->status_host[slot] = 0;
    q.slot = slot;
    q.ws_off = off;
    q.ws_bytes = ws;
    q.ev = ev;
    q.done_cells = 0;
    q.stream = -1;  // its first slice waits for dispatch
    q.state = BZ_REQ_ADMITTED;
    q.t_admit = now_ns();
    cp->inflight += 1;
    cp->last_use = q.t_admit;
    s->inflight.push_back(id);
    admitted.push_back(c.pos);
  }
  if (!progress) return false;
  // bypass counts of the requests still queued, then drop the others from the queue
  for (size_t qi = 0; qi < window; ++qi) {
    if (gone[qi]) continue;
    for (size_t a : admitted)
      if (a > qi) s->reqs[s->queue[qi]].bypassed += 1;
  }
  std::deque<uint64_t> rest;
  for (size_t qi = 0; qi < s->queue.size(); ++qi)
    if (qi >= window || !gone[qi]) rest.push_back(s->queue[qi]);
  s->queue.swap(rest);
  return true;
}

void scheduler(bz_server* s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    reap(s);
    const uint64_t seen = s->gen;
    admit(s);
    dispatch(s);
    trim_host_plans(s);
    if (s->stop && s->queue.empty() && s->inflight.empty()) break;
    if (s->inflight.empty()) {
      // nothing on the GPU: sleep until a submission, a finished build or stop
      // (every queued request that could be admitted now has been)
      s->cv.wait(lk, [s, seen] { return s->gen != seen; });
    } else {
      lk.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(20));
      lk.lock();
    }
  }
}

}  // namespace

extern "C" {

bz_status bz_server_create(const bz_server_desc* d, bz_server** out) {
  bz::clear_error();
  if (!d || !out) return bz::fail(BZ_ERR_ARG, "bz_server_create: null argument");
  *out = nullptr;
  if (!d->arena_dev || d->arena_bytes < kAlign) return bz::fail(BZ_ERR_ARG, "bz_server_create: arena missing or too small");
  if (uintptr_t(d->arena_dev) & (kAlign - 1)) return bz::fail(BZ_ERR_ARG, "bz_server_create: arena must be 256-byte aligned");
  if (d->max_inflight < 1 || d->n_streams < 1 || d->n_streams > 16 || d->max_queue < 1 || d->slice_cells < 0)
    return bz::fail(BZ_ERR_ARG, "bz_server_create: need max_inflight >= 1, 1 <= n_streams <= 16, max_queue >= 1, "
                    "slice_cells >= 0");
  auto s = std::make_unique<bz_server>();
  s->d = *d;
  s->arena.init(d->arena_dev, d->arena_bytes);
  if (hipGetDevice(&s->device) != hipSuccess) return bz::fail(BZ_ERR_DEVICE, "bz_server_create: no device");
  for (int i = 0; i < d->n_streams + 1; ++i) {
    hipStream_t st = nullptr;
    const hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e != hipSuccess) {
      for (auto x : s->streams) (void)hipStreamDestroy(x);
      return bz::fail(BZ_ERR_DEVICE, "bz_server_create: %s", hipGetErrorString(e));
    }
    if (i < d->n_streams) s->streams.push_back(st);
    else s->upload = st;
  }
  s->stream_load.assign(s->streams.size(), 0.0);
  s->stream_depth.assign(s->streams.size(), 0);
  if (hipHostMalloc(reinterpret_cast<void**>(&s->status_host), sizeof(int32_t) * size_t(d->max_inflight),
                    hipHostMallocDefault) != hipSuccess) {
    for (auto x : s->streams) (void)hipStreamDestroy(x);
    if (s->upload) (void)hipStreamDestroy(s->upload);
    return bz::fail(BZ_ERR_DEVICE, "bz_server_create: pinned status buffer");
  }
  for (int i = d->max_inflight - 1; i >= 0; --i) s->free_slots.push_back(i);
  bz_server* raw = s.release();
  raw->th = std::thread(scheduler, raw);
  raw->builder = std::thread(builder, raw);
  *out = raw;
  return BZ_OK;
}

bz_status bz_serve_submit(bz_server* s, const bz_request* r, uint64_t* ticket) {
  bz::clear_error();
  if (!s || !r || !ticket) return bz::fail(BZ_ERR_ARG, "bz_serve_submit: null argument");
  if (r->ncells < 0) return bz::fail(BZ_ERR_ARG, "bz_serve_submit: ncells < 0");
  if (r->ncells > 0 && (!r->f || !r->q)) return bz::fail(BZ_ERR_ARG, "bz_serve_submit: null f or q");
  if (r->f_dtype != BZ_FP32 && r->f_dtype != BZ_FP64) return bz::fail(BZ_ERR_ARG, "bz_serve_submit: bad f_dtype");
  if ((r->flags & BZ_SCATTER) && !r->idx) return bz::fail(BZ_ERR_ARG, "bz_serve_submit: BZ_SCATTER needs idx");
  if (r->plan.dir_kind == BZ_DIRS_EXPLICIT && (!r->plan.dirs || !r->plan.weights || r->plan.m < 1 || r->plan.m > 512))
    return bz::fail(BZ_ERR_ARG, "bz_serve_submit: explicit rule needs dirs and weights");
  std::lock_guard<std::mutex> g(s->mu);
  if (s->stop) return bz::fail(BZ_ERR_STATE, "bz_serve_submit: server is shutting down");
  if (int(s->queue.size()) >= s->d.max_queue) return BZ_AGAIN;
  Req q;
  q.ticket = s->next_ticket++;
  q.r = *r;
  q.slice = slice_cells(s->d, r->plan);
  q.key = make_key(r->plan, std::min(r->ncells, q.slice), s->arena.bytes);
  q.t_submit = now_ns();
  if (s->submitted == 0) s->t_first_submit = q.t_submit;
  s->submitted += 1;
  *ticket = q.ticket;
  s->queue.push_back(q.ticket);
  s->reqs.emplace(q.ticket, std::move(q));
  s->gen += 1;
  s->cv.notify_one();
  return BZ_OK;
}

bz_status bz_serve_poll(bz_server* s, uint64_t ticket, bz_result* out) {
  bz::clear_error();
  if (!s || !out) return bz::fail(BZ_ERR_ARG, "bz_serve_poll: null argument");
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return bz::fail(BZ_ERR_ARG, "bz_serve_poll: unknown or already collected ticket %llu", (unsigned long long)ticket);
  const Req& q = it->second;
  out->state = q.state;
  out->err = q.err;
  out->t_submit_ns = q.t_submit;
  out->t_admit_ns = q.t_admit;
  out->t_done_ns = q.t_done;
  if (q.state == BZ_REQ_DONE || q.state == BZ_REQ_FAILED) {
    s->reqs.erase(it);
    return BZ_OK;
  }
  return BZ_AGAIN;
}

bz_status bz_server_stats_ex(bz_server* s, bz_server_stats_t* out) {
  bz::clear_error();
  if (!s || !out) return bz::fail(BZ_ERR_ARG, "bz_server_stats_ex: null argument");
  std::lock_guard<std::mutex> g(s->mu);
  std::memset(out, 0, sizeof *out);
  out->submitted = s->submitted;
  out->completed = s->completed;
  out->failed = s->failed;
  out->queued = int32_t(s->queue.size());
  out->inflight = int32_t(s->inflight.size());
  out->plans_cached = int32_t(s->plans.size());
  out->arena_used = s->arena.used;
  out->arena_peak = s->arena.peak;
  if (!s->lat_ms.empty()) {
    std::vector<double> v = s->lat_ms;
    std::sort(v.begin(), v.end());
    auto pct = [&](double p) {
      const size_t i = size_t(std::min<double>(double(v.size() - 1), std::ceil(p * double(v.size())) - 1.0));
      return v[i];
    };
    out->p50_ms = pct(0.50);
    out->p99_ms = pct(0.99);
  }
  if (s->t_last_done > s->t_first_submit)
    out->cells_per_s = double(s->cells_done) / (double(s->t_last_done - s->t_first_submit) * 1e-9);
  return BZ_OK;
}

bz_status bz_server_stats(bz_server* s, double* p50_ms, double* p99_ms, double* cells_per_s) {
  bz_server_stats_t st;
  const bz_status e = bz_server_stats_ex(s, &st);
  if (e != BZ_OK) return e;
  if (p50_ms) *p50_ms = st.p50_ms;
  if (p99_ms) *p99_ms = st.p99_ms;
  if (cells_per_s) *cells_per_s = st.cells_per_s;
  return BZ_OK;
}

bz_status bz_server_destroy(bz_server* s) {
  bz::clear_error();
  if (!s) return BZ_OK;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
    s->gen += 1;
  }
  s->cv.notify_all();
  if (s->th.joinable()) s->th.join();  // drains every request (the builder still builds for it)
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->builder_stop = true;
  }
  s->build_cv.notify_all();
  if (s->builder.joinable()) s->builder.join();
  for (auto& c : s->plans) free_plan(c.get());
  for (auto e : s->event_pool) (void)hipEventDestroy(e);
  for (auto x : s->streams) (void)hipStreamDestroy(x);
  if (s->upload) (void)hipStreamDestroy(s->upload);
  if (s->status_host) (void)hipHostFree(s->status_host);
  delete s;
  return BZ_OK;
}

}  // extern "C"
