// Request server: a native scheduler over a fixed set of device streams.
//
// Submissions go into a FIFO queue.  A scheduler thread admits requests
// first-fit: whenever a slot (stream) is free and a queued request's working
// memory fits what is left of the HBM budget, it allocates that memory
// stream-ordered, enqueues the request's whole step loop on the slot's
// stream, frees the memory stream-ordered behind it and appends a host
// callback that stamps the completion time.  Retiring a request returns its
// slot and budget at once, so requests arriving while others run are
// admitted as soon as room appears and their kernels overlap on the device.
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
};

struct SSlot;

}  // namespace

struct ffs_server_s {
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

}  // namespace

extern "C" {

void ffs_server_default_options(ffs_server_options* o) {
  if (!o) return;
  o->slots = 4;
  o->reserved = 0;
  o->hbm_budget = 0;
}

ffs_status ffs_server_create(ffs_server_t* out, const ffs_server_options* opt) {
  if (!out) return (ffs_status)set_error(FFS_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  ffs_server_options o;
  ffs_server_default_options(&o);
  if (opt) o = *opt;
  if (o.slots < 1 || o.slots > 32 || o.reserved != 0)
    return (ffs_status)set_error(FFS_ERR_INVALID_ARG, "slots must be in 1..32");
  ffs_server_s* s = new ffs_server_s();
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
