// Request server: a native scheduler thread in front of the device.
//
// Submissions go into a FIFO queue; the scheduler admits requests first fit
// (a request whose working memory fits what is left of the HBM budget may
// pass a larger one that does not), allocates that memory stream-ordered at
// admission and frees it stream-ordered when the request is done; a host
// callback behind the request's last device work stamps its completion.
//
// Grouped mode (continuous batching): running requests are instances of one
// resident group table.  Each round the scheduler retires instances that
// reached their last step (copy-out, counters, free), admits queued
// requests into free table entries (first step with the ordinary launches),
// uploads the table and work lists from a pinned staging ring, and enqueues
// `ticks` lockstep steps -- one launch per phase for every instance, each at
// its own step.  Every active instance advances exactly one step per tick,
// so the host tracks each instance's step without reading it back.  At most
// two rounds are in flight.
//
// Streams mode: every running request has a stream of its own and runs its
// whole step loop there.
#include <hip/hip_runtime.h>
#include <string.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/ffs.h"
#include "ffs_internal.h"

using namespace ffsk;

namespace {

using Clock = std::chrono::steady_clock;

struct Req {
  uint64_t id = 0;
  ffs_plan_s* plan = nullptr;
  int64_t n_keep = 0, n = 0;
  uint64_t seed = 0, first = 0;
  int32_t* x = nullptr;
  double* ld = nullptr;
  size_t bytes = 0;
  int s_chunk = 0;
  int state = FFS_REQ_QUEUED;
  int status = FFS_OK;
  double t_submit = 0, t_admit = 0, t_done = 0;
  int64_t flagged = 0, changed = 0;
  // grouped mode: completion stamped by the host callback
  ffs_server_s* srv = nullptr;
  std::atomic<int> cb_done{0};
  std::atomic<double> cb_t{0.0};
  int stat_slot = -1;
};

struct SSlot;
struct GroupRT;

}  // namespace

struct ffs_server_s {
  int mode = FFS_SERVE_GROUPED;
  GroupRT* grp = nullptr;
  int device = 0;
  size_t budget = 0, used = 0;
  std::vector<SSlot*> slots;
  std::deque<Req*> queue;
  std::unordered_map<uint64_t, Req*> reqs;
  uint64_t next_id = 1;
  std::mutex mu;
  std::condition_variable cv;
  std::thread th;
  bool stop = false;
  Clock::time_point t0;
  double now() const {
    return std::chrono::duration<double>(Clock::now() - t0).count();
  }
};

namespace {

struct SSlot {
  ffs_server_s* srv = nullptr;
  hipStream_t st = nullptr;
  unsigned long long* pinned = nullptr;  // [0] flagged [1] changed [2] ctl words
  Req* r = nullptr;                      // request in flight (guarded by mu)
  std::atomic<int> done{0};
  std::atomic<double> t_done{0.0};
};

void on_done(void* arg) {  // runs on the runtime's callback thread
  SSlot* sl = static_cast<SSlot*>(arg);
  sl->t_done.store(sl->srv->now());
  sl->done.store(1);
  sl->srv->cv.notify_all();
}

// Enqueue one admitted request on its slot's stream (no lock held).  Returns
// the request's status; on failure nothing of it remains in flight.
int launch(SSlot* sl, Req* r) {
  void* mem = nullptr;
  if (hipMallocAsync(&mem, r->bytes, sl->st) != hipSuccess) return FFS_ERR_OUT_OF_MEMORY;
  const int st = run_request(r->plan, mem, r->s_chunk, r->seed, r->first, r->n,
                             (int)r->n_keep, r->x, r->ld, sl->st, sl->pinned);
  (void)hipFreeAsync(mem, sl->st);
  if (st == FFS_OK && hipLaunchHostFunc(sl->st, on_done, sl) == hipSuccess) return FFS_OK;
  (void)hipStreamSynchronize(sl->st);
  return st == FFS_OK ? FFS_ERR_HIP : st;
}

void scheduler(ffs_server_s* s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  std::vector<std::pair<SSlot*, Req*>> admitted;
  while (true) {
    bool changed = false;
    for (SSlot* sl : s->slots) {  // retire finished requests
      if (!sl->r || !sl->done.load()) continue;
      Req* r = sl->r;
      r->t_done = sl->t_done.load();
      r->flagged = (int64_t)sl->pinned[0];
      r->changed = (int64_t)sl->pinned[1];
      const uint32_t dev_status = (uint32_t)(sl->pinned[2] >> 32);
      if (dev_status & DEV_NUMERICAL) r->status = FFS_ERR_NUMERICAL;
      r->state = FFS_REQ_DONE;
      s->used -= r->bytes;
      sl->r = nullptr;
      changed = true;
    }
    if (s->stop) {
      bool busy = false;
      for (SSlot* sl : s->slots) busy |= sl->r != nullptr;
      if (!busy) break;
    } else {
      admitted.clear();
      for (SSlot* sl : s->slots) {  // admit first-fit
        if (sl->r) continue;
        auto it = s->queue.begin();
        while (it != s->queue.end() && s->used + (*it)->bytes > s->budget) ++it;
        if (it == s->queue.end()) break;
        Req* r = *it;
        s->queue.erase(it);
        r->state = FFS_REQ_RUNNING;
        r->t_admit = s->now();
        s->used += r->bytes;
        sl->r = r;
        sl->done.store(0);
        admitted.emplace_back(sl, r);
      }
      if (!admitted.empty()) {
        lk.unlock();  // enqueueing a long step loop must not block submit/poll
        std::vector<int> st(admitted.size());
        for (size_t i = 0; i < admitted.size(); ++i)
          st[i] = launch(admitted[i].first, admitted[i].second);
        lk.lock();
        for (size_t i = 0; i < admitted.size(); ++i) {
          if (st[i] == FFS_OK) continue;
          Req* r = admitted[i].second;
          r->status = st[i];
          r->state = FFS_REQ_DONE;
          r->t_done = s->now();
          s->used -= r->bytes;
          admitted[i].first->r = nullptr;
        }
        changed = true;
      }
    }
    if (changed) s->cv.notify_all();
    s->cv.wait_for(lk, std::chrono::microseconds(200));
  }
  s->cv.notify_all();
}

// ------------------------------------------------------------ grouped ----
struct Member {
  Req* r = nullptr;
  PlanView pv;
  Work w;
  void* mem = nullptr;
  int t = 0;  // step the next tick performs (mirrors the device counter)
};

struct GroupRT {
  int cap = 0, ticks = 0;
  hipStream_t st = nullptr;
  GInst* dev_inst = nullptr;  // [cap]
  int* dev_lists = nullptr;   // kGroupLists lists x (cap ids + cap + 1 prefix entries)
  static constexpr int RING = 3;
  char* pin[RING] = {nullptr, nullptr, nullptr};
  hipEvent_t pin_ev[RING] = {nullptr, nullptr, nullptr};
  int ring = 0;
  std::deque<hipEvent_t> inflight, spare;
  unsigned long long* stats_pin = nullptr;  // [4*cap][4]: flagged, changed, ctl
  std::vector<int> free_stats;
  std::vector<Member*> members;
  std::vector<Req*> finishing;
  size_t table_bytes() const {
    return (size_t)cap * sizeof(GInst) + (size_t)kGroupLists * (2 * cap + 1) * sizeof(int);
  }
};

void on_req_done(void* arg) {  // runtime callback thread: no HIP calls
  Req* r = static_cast<Req*>(arg);
  r->cb_t.store(r->srv->now());
  r->cb_done.store(1);
  r->srv->cv.notify_all();
}

// Enqueue the end of a finished instance: copy-out, its counters, free.
void retire_member(ffs_server_s* s, GroupRT* g, Member* m) {
  Req* r = m->r;
  launch_copy_out(m->pv.d, m->w, (int)r->n, (int)r->n_keep, r->x, r->ld, g->st);
  if (!g->free_stats.empty()) {
    r->stat_slot = g->free_stats.back();
    g->free_stats.pop_back();
    unsigned long long* dst = g->stats_pin + 4 * (size_t)r->stat_slot;
    (void)hipMemcpyAsync(dst, m->w.counters, 16, hipMemcpyDeviceToHost, g->st);
    (void)hipMemcpyAsync(dst + 2, m->w.ctl, 8, hipMemcpyDeviceToHost, g->st);
  }
  (void)hipFreeAsync(m->mem, g->st);
  s->used -= r->bytes;
  if (hipLaunchHostFunc(g->st, on_req_done, r) != hipSuccess) {
    (void)hipStreamSynchronize(g->st);
    on_req_done(r);
  }
  g->finishing.push_back(r);
}

void group_scheduler(ffs_server_s* s) {
  (void)hipSetDevice(s->device);
  GroupRT* g = s->grp;
  std::unique_lock<std::mutex> lk(s->mu);
  while (true) {
    bool changed = false;
    // completions reported by the callbacks
    for (size_t k = 0; k < g->finishing.size();) {
      Req* r = g->finishing[k];
      if (!r->cb_done.load()) {
        ++k;
        continue;
      }
      r->t_done = r->cb_t.load();
      if (r->stat_slot >= 0) {
        const unsigned long long* src = g->stats_pin + 4 * (size_t)r->stat_slot;
        r->flagged = (int64_t)src[0];
        r->changed = (int64_t)src[1];
        if ((uint32_t)(src[2] >> 32) & DEV_NUMERICAL) r->status = FFS_ERR_NUMERICAL;
        g->free_stats.push_back(r->stat_slot);
      }
      r->state = FFS_REQ_DONE;
      g->finishing[k] = g->finishing.back();
      g->finishing.pop_back();
      changed = true;
    }
    // instances that performed their last step
    int active = 0;
    for (Member*& m : g->members) {
      if (!m) continue;
      if (m->t >= m->r->n_keep) {
        retire_member(s, g, m);
        delete m;
        m = nullptr;
        changed = true;
      } else {
        ++active;
      }
    }
    if (s->stop && active == 0 && g->finishing.empty()) break;
    // admissions, first fit
    if (!s->stop) {
      for (size_t i = 0; i < g->members.size() && !s->queue.empty(); ++i) {
        if (g->members[i]) continue;
        auto it = s->queue.begin();
        while (it != s->queue.end() && s->used + (*it)->bytes > s->budget) ++it;
        if (it == s->queue.end()) break;
        Req* r = *it;
        s->queue.erase(it);
        Member* m = new Member();
        m->r = r;
        m->pv = plan_view(r->plan);
        if (hipMallocAsync(&m->mem, r->bytes, g->st) != hipSuccess) {
          r->status = FFS_ERR_OUT_OF_MEMORY;
          r->state = FFS_REQ_DONE;
          r->t_done = s->now();
          delete m;
          changed = true;
          continue;
        }
        carve(m->pv.d, static_cast<char*>(m->mem), (int)((r->n + SAMPLE_PAD - 1) / SAMPLE_PAD * SAMPLE_PAD),
              &m->w);
        start_instance(m->pv, m->w, (int)r->n, (int)r->n_keep, r->seed, r->first, g->st);
        r->state = FFS_REQ_RUNNING;
        r->t_admit = s->now();
        s->used += r->bytes;
        g->members[i] = m;
        ++active;
        changed = true;
      }
    }
    if (changed) s->cv.notify_all();
    if (active == 0) {
      s->cv.wait_for(lk, std::chrono::microseconds(200));
      continue;
    }
    // table and lists for this round
    const int k = g->ring;
    g->ring = (g->ring + 1) % GroupRT::RING;
    (void)hipEventSynchronize(g->pin_ev[k]);
    char* hst = g->pin[k];
    GInst* tab = reinterpret_cast<GInst*>(hst);
    int* lists = reinterpret_cast<int*>(hst + (size_t)g->cap * sizeof(GInst));
    std::vector<int> ids[kGroupLists], pre[kGroupLists];
    int maxN[2] = {1, 1};
    for (int i = 0; i < g->cap; ++i) {
      Member* m = g->members[i];
      if (!m) {
        tab[i].t = 0;
        tab[i].n_keep = 0;  // never active
        continue;
      }
      tab[i] = make_ginst(m->pv, m->w, (int)m->r->n, (int)m->r->n_keep, m->r->seed, m->r->first);
      tab[i].t = m->t;
      int items[kGroupLists];
      group_items(m->pv.d, (int)m->r->n, items);
      for (int q = 0; q < kGroupLists; ++q) {
        if (items[q] <= 0) continue;
        if (pre[q].empty()) pre[q].push_back(0);
        ids[q].push_back(i);
        pre[q].push_back(pre[q].back() + items[q]);
      }
      const int c = m->pv.d.cplx ? 1 : 0;
      maxN[c] = m->pv.d.N > maxN[c] ? m->pv.d.N : maxN[c];
    }
    GList gl[kGroupLists];
    for (int q = 0; q < kGroupLists; ++q) {
      int* h = lists + (size_t)q * (2 * g->cap + 1);
      int* dv = g->dev_lists + (size_t)q * (2 * g->cap + 1);
      const int ni = (int)ids[q].size();
      for (int j = 0; j < ni; ++j) h[j] = ids[q][j];
      for (int j = 0; j <= ni && !pre[q].empty(); ++j) h[g->cap + j] = pre[q][j];
      gl[q].ids = dv;
      gl[q].pre = dv + g->cap;
      gl[q].n = ni;
      gl[q].total = ni ? pre[q].back() : 0;
    }
    (void)hipMemcpyAsync(g->dev_inst, hst, g->table_bytes(), hipMemcpyHostToDevice, g->st);
    (void)hipEventRecord(g->pin_ev[k], g->st);
    for (int q = 0; q < g->ticks; ++q) launch_tick(g->dev_inst, gl, maxN, g->cap, g->st);
    for (Member* m : g->members)
      if (m) m->t = (m->t + g->ticks < m->r->n_keep) ? m->t + g->ticks : (int)m->r->n_keep;
    hipEvent_t ev;
    if (!g->spare.empty()) {
      ev = g->spare.front();
      g->spare.pop_front();
    } else {
      (void)hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    }
    (void)hipEventRecord(ev, g->st);
    g->inflight.push_back(ev);
    if (g->inflight.size() > 2) {  // bound the work queued ahead of the device
      hipEvent_t old = g->inflight.front();
      g->inflight.pop_front();
      lk.unlock();
      (void)hipEventSynchronize(old);
      lk.lock();
      g->spare.push_back(old);
    }
  }
  s->cv.notify_all();
}

ffs_status group_create(ffs_server_s* s, int cap, int ticks) {
  GroupRT* g = new GroupRT();
  g->cap = cap;
  g->ticks = ticks;
  g->members.assign(cap, nullptr);
  s->grp = g;
  if (hipStreamCreateWithFlags(&g->st, hipStreamNonBlocking) != hipSuccess ||
      hipMalloc((void**)&g->dev_inst, g->table_bytes()) != hipSuccess ||
      hipHostMalloc((void**)&g->stats_pin, (size_t)4 * cap * 32, 0) != hipSuccess)
    return FFS_ERR_HIP;
  g->dev_lists = reinterpret_cast<int*>(reinterpret_cast<char*>(g->dev_inst) + (size_t)cap * sizeof(GInst));
  for (int i = 0; i < GroupRT::RING; ++i)
    if (hipHostMalloc((void**)&g->pin[i], g->table_bytes(), 0) != hipSuccess ||
        hipEventCreateWithFlags(&g->pin_ev[i], hipEventDisableTiming) != hipSuccess)
      return FFS_ERR_HIP;
  for (int i = 4 * cap - 1; i >= 0; --i) g->free_stats.push_back(i);
  return FFS_OK;
}

void group_destroy(ffs_server_s* s) {
  GroupRT* g = s->grp;
  if (!g) return;
  if (g->st) (void)hipStreamSynchronize(g->st);
  for (hipEvent_t e : g->inflight) (void)hipEventDestroy(e);
  for (hipEvent_t e : g->spare) (void)hipEventDestroy(e);
  for (int i = 0; i < GroupRT::RING; ++i) {
    if (g->pin[i]) (void)hipHostFree(g->pin[i]);
    if (g->pin_ev[i]) (void)hipEventDestroy(g->pin_ev[i]);
  }
  if (g->stats_pin) (void)hipHostFree(g->stats_pin);
  if (g->dev_inst) (void)hipFree(g->dev_inst);
  if (g->st) (void)hipStreamDestroy(g->st);
  delete g;
  s->grp = nullptr;
}

}  // namespace

extern "C" {

void ffs_server_default_options(ffs_server_options* o) {
  if (!o) return;
  o->mode = FFS_SERVE_GROUPED;
  o->slots = 4;
  o->hbm_budget = 0;
  o->capacity = 128;
  o->ticks = 8;
}

ffs_status ffs_server_create(ffs_server_t* out, const ffs_server_options* opt) {
  if (!out) return (ffs_status)set_error(FFS_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  ffs_server_options o;
  ffs_server_default_options(&o);
  if (opt) o = *opt;
  if ((o.mode != FFS_SERVE_GROUPED && o.mode != FFS_SERVE_STREAMS) || o.slots < 1 ||
      o.slots > 32 || o.capacity < 1 || o.capacity > 1024 || o.ticks < 1 || o.ticks > 256)
    return (ffs_status)set_error(FFS_ERR_INVALID_ARG, "bad server options");
  ffs_server_s* s = new ffs_server_s();
  s->mode = o.mode;
  s->t0 = Clock::now();
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return (ffs_status)set_error(FFS_ERR_HIP, "no HIP device");
  }
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
    delete s;
    return (ffs_status)set_error(FFS_ERR_HIP, "hipMemGetInfo failed");
  }
  s->budget = o.hbm_budget ? o.hbm_budget : free_b / 2;
  if (s->mode == FFS_SERVE_GROUPED) {
    if (group_create(s, o.capacity, o.ticks) != FFS_OK) {
      group_destroy(s);
      delete s;
      return (ffs_status)set_error(FFS_ERR_HIP, "group runtime creation failed");
    }
    s->th = std::thread(group_scheduler, s);
    *out = s;
    return FFS_OK;
  }
  for (int i = 0; i < o.slots; ++i) {
    SSlot* sl = new SSlot();
    sl->srv = s;
    if (hipStreamCreateWithFlags(&sl->st, hipStreamNonBlocking) != hipSuccess ||
        hipHostMalloc((void**)&sl->pinned, 64, 0) != hipSuccess) {
      if (sl->st) (void)hipStreamDestroy(sl->st);
      delete sl;
      for (SSlot* q : s->slots) {
        (void)hipStreamDestroy(q->st);
        (void)hipHostFree(q->pinned);
        delete q;
      }
      delete s;
      return (ffs_status)set_error(FFS_ERR_HIP, "stream or pinned buffer creation failed");
    }
    memset(sl->pinned, 0, 64);
    s->slots.push_back(sl);
  }
  s->th = std::thread(scheduler, s);
  *out = s;
  return FFS_OK;
}

ffs_status ffs_server_submit(ffs_server_t sv, ffs_plan_t p, int64_t n_keep,
                             uint64_t seed, uint64_t first_sample,
                             int64_t n_samples, int32_t* x_dev,
                             double* logdet_dev, uint64_t* ticket) {
  ffs_server_s* s = sv;
  if (!s || !p || !x_dev || !ticket)
    return (ffs_status)set_error(FFS_ERR_INVALID_ARG, "NULL argument");
  if (plan_path(p) != FFS_PATH_BATCHED)
    return (ffs_status)set_error(FFS_ERR_INVALID_ARG, "the server runs batched-path plans only");
  if (plan_device(p) != s->device)
    return (ffs_status)set_error(FFS_ERR_INVALID_ARG, "plan is on another device");
  const Dims& d = plan_dims(p);
  if (n_keep < 1 || n_keep > d.N || n_samples < 1)
    return (ffs_status)set_error(FFS_ERR_INVALID_ARG, "n_keep or n_samples out of range");
  if (logdet_dev && n_keep != d.N)
    return (ffs_status)set_error(FFS_ERR_INVALID_ARG, "logdet needs n_keep = N");
  if (s->mode == FFS_SERVE_GROUPED) {
    const PlanView pv = plan_view(p);
    if (n_samples > pv.max_batch)
      return (ffs_status)set_error(FFS_ERR_INVALID_ARG, "grouped serving: n_samples above the plan's max_batch");
  }
  const double t_submit = s->now();
  Req* r = new Req();
  r->plan = p;
  r->n_keep = n_keep;
  r->n = n_samples;
  r->seed = seed;
  r->first = first_sample;
  r->x = x_dev;
  r->ld = logdet_dev;
  r->bytes = request_bytes(p, n_samples, &r->s_chunk);
  r->srv = s;
  if (r->bytes > s->budget) {
    delete r;
    return (ffs_status)set_error(FFS_ERR_OUT_OF_MEMORY, "request working memory exceeds the server budget");
  }
  {
    std::lock_guard<std::mutex> g(s->mu);
    if (s->stop) {
      delete r;
      return (ffs_status)set_error(FFS_ERR_INVALID_ARG, "server is shutting down");
    }
    r->id = s->next_id++;
    r->t_submit = t_submit;
    s->queue.push_back(r);
    s->reqs[r->id] = r;
    *ticket = r->id;
  }
  s->cv.notify_all();
  return FFS_OK;
}

ffs_status ffs_server_poll(ffs_server_t sv, uint64_t ticket, int32_t timeout_ms,
                           ffs_request_info* info) {
  ffs_server_s* s = sv;
  if (!s) return (ffs_status)set_error(FFS_ERR_INVALID_ARG, "server is NULL");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return (ffs_status)set_error(FFS_ERR_INVALID_ARG, "unknown ticket");
  Req* r = it->second;
  if (timeout_ms < 0)
    s->cv.wait(lk, [&] { return r->state == FFS_REQ_DONE; });
  else if (timeout_ms > 0)
    s->cv.wait_for(lk, std::chrono::milliseconds(timeout_ms),
                   [&] { return r->state == FFS_REQ_DONE; });
  if (info) {
    info->state = r->state;
    info->status = r->status;
    info->t_submit = r->t_submit;
    info->t_admit = r->t_admit;
    info->t_done = r->t_done;
    info->draws = r->n * r->n_keep;
    info->flagged = r->flagged;
    info->changed = r->changed;
  }
  if (r->state == FFS_REQ_DONE) {
    s->reqs.erase(it);
    delete r;
  }
  return FFS_OK;
}

ffs_status ffs_server_destroy(ffs_server_t sv) {
  ffs_server_s* s = sv;
  if (!s) return (ffs_status)set_error(FFS_ERR_INVALID_ARG, "server is NULL");
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
    for (Req* r : s->queue) {
      s->reqs.erase(r->id);
      delete r;
    }
    s->queue.clear();
  }
  s->cv.notify_all();
  s->th.join();
  group_destroy(s);
  for (SSlot* sl : s->slots) {
    (void)hipStreamSynchronize(sl->st);
    (void)hipStreamDestroy(sl->st);
    (void)hipHostFree(sl->pinned);
    delete sl;
  }
  for (auto& kv : s->reqs) delete kv.second;
  delete s;
  return FFS_OK;
}

}  // extern "C"
