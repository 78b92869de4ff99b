// Grouped executor: many instances (plan, sample count, n_keep) advanced in
// lockstep with one launch per phase for all of them.
//
// Host side: validates the instances, lays out one stream-ordered
// allocation holding every instance's working memory, uploads the instance
// table (argument blocks of every phase plus the device-side step counter)
// and the work-item lists, runs each instance's first factor step with the
// ordinary launches, then issues ticks -- contraction, draw, redraw, factor,
// advance -- either directly or as a captured hipGraph of up to 16 ticks
// replayed until the longest instance is done, and finally copies every
// instance's draws out.
#include <hip/hip_runtime.h>
#include <string.h>

#include <mutex>
#include <vector>

#include "../../include/ffs.h"
#include "ffs_internal.h"

using namespace ffsk;

namespace {

inline int64_t rup(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

// Pinned staging of the tables, reused across calls once the previous
// upload has executed; graph objects are destroyed once their last replay
// has completed.
struct Staging {
  std::mutex mu;
  void* host = nullptr;
  size_t cap = 0;
  hipEvent_t uploaded = nullptr;
  int device = -1;
  hipStream_t st = nullptr;  // internal stream (capture needs a non-legacy stream)
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  struct Dead {
    hipGraphExec_t exec;
    hipGraph_t graph;
    hipEvent_t done;
  };
  std::vector<Dead> dead;
};
Staging g_stage;

struct ListBuild {
  std::vector<int> ids, pre{0};
  void add(int id, int items) {
    if (items <= 0) return;
    ids.push_back(id);
    pre.push_back(pre.back() + items);
  }
};

}  // namespace

namespace ffsk {

GInst make_ginst(const PlanView& pv, const Work& w, int S, int n_keep,
                 uint64_t seed, uint64_t first) {
  GInst g;
  g.wa = make_wargs(pv.d, w, pv.ubulk);
  g.uh = pv.d.bf16 ? static_cast<const uint16_t*>(pv.ubf) : nullptr;
  g.ul = pv.d.bf16 ? g.uh + (size_t)pv.d.Kg * pv.d.L_pad : nullptr;
  g.da = make_dargs(pv.d, w, S, seed, first, pv.delta, pv.coef, 0);
  g.ra = make_rargs(pv.d, w, pv.u64t, seed, first);
  g.fa = make_fargs(pv.d, w, pv.u64, n_keep, seed, first);
  g.t = 0;
  g.n_keep = n_keep;
  g.S = S;
  g.cplx = pv.d.cplx;
  return g;
}

void start_instance(const PlanView& pv, const Work& w, int S, int n_keep,
                    uint64_t seed, uint64_t first, hipStream_t st) {
  (void)hipMemsetAsync(w.gam, 0, (size_t)w.S_pad * pv.d.Kg * 4, st);
  (void)hipMemsetAsync(w.ctl, 0, 256, st);
  (void)hipMemsetAsync(w.counters, 0, 256, st);
  launch_init(pv.d, w, S, st);
  launch_factor(pv.d, w, pv.u64, S, -1, 0, n_keep, seed, first, st);
}

// Work items of one instance in each list (weights real / complex per tile,
// redraw product real / complex, factor real / complex, draw); the redraw of
// flagged draws runs inside the factor launch.
void group_items(const Dims& d, int S, int items[kGroupLists]) {
  const int c = d.cplx ? 1 : 0;
  for (int k = 0; k < kGroupLists; ++k) items[k] = 0;
  const int s_round = (S + SAMPLE_PAD - 1) / SAMPLE_PAD * SAMPLE_PAD;
  if (d.bf16) {
    items[11 + c] = weights_bf16_group_items(d, S);
  } else {
    // grouped launches run the 32-wide-chunk variant of the chosen tile
    // (the same results bit for bit)
    const int v = kTiles[tile_choice(d, s_round)].base;
    items[c ? 4 + v : v] = weights_group_items(d, S, v);
  }
  items[6 + c] = repair_group_items(d, S);
  items[8 + c] = S;
  items[10] = S;
}

void launch_tick(GInst* inst, const GList* gl, const int* maxN, int n_inst, hipStream_t st) {
  for (int v = 0; v < 4; ++v) launch_weights_group(inst, gl[v], false, v, st);
  for (int v = 0; v < 2; ++v) launch_weights_group(inst, gl[4 + v], true, v, st);
  launch_weights_bf16_group(inst, gl[11], false, st);
  launch_weights_bf16_group(inst, gl[12], true, st);
  launch_draw_group(inst, gl[10], st);
  launch_repair_group(inst, gl[6], false, st);
  launch_repair_group(inst, gl[7], true, st);
  launch_factor_group(inst, gl[8], false, maxN[0], st);
  launch_factor_group(inst, gl[9], true, maxN[1], st);
  launch_advance(inst, n_inst, st);
}

}  // namespace ffsk

extern "C" ffs_status ffs_sample_group(const ffs_instance* in, int32_t n,
                                       int32_t flags, ffs_stats_t* stats,
                                       void* stream) {
  if (n < 0 || (n > 0 && !in)) return (ffs_status)set_error(FFS_ERR_INVALID_ARG, "bad instance array");
  if (flags & ~FFS_GROUP_GRAPH) return (ffs_status)set_error(FFS_ERR_INVALID_ARG, "unknown flags");
  if (n == 0) return FFS_OK;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return (ffs_status)set_error(FFS_ERR_HIP, "no HIP device");
  std::vector<PlanView> pv(n);
  for (int i = 0; i < n; ++i) {
    const ffs_instance& q = in[i];
    if (!q.plan || !q.x_dev) return (ffs_status)set_error(FFS_ERR_INVALID_ARG, "NULL plan or x_dev");
    if (plan_path(q.plan) != FFS_PATH_BATCHED || plan_device(q.plan) != dev)
      return (ffs_status)set_error(FFS_ERR_INVALID_ARG, "instances need batched-path plans on the current device");
    pv[i] = plan_view(q.plan);
    if (q.n_keep < 1 || q.n_keep > pv[i].d.N || q.n_samples < 1 || q.n_samples > pv[i].max_batch)
      return (ffs_status)set_error(FFS_ERR_INVALID_ARG, "n_keep or n_samples out of range");
    if (q.logdet_dev && q.n_keep != pv[i].d.N)
      return (ffs_status)set_error(FFS_ERR_INVALID_ARG, "logdet needs n_keep = N");
  }

  // ---- layout: tables, then per-instance working memory -------------------
  ListBuild lists_b[kGroupLists];
  int maxN[2] = {1, 1}, T_max = 0;
  for (int i = 0; i < n; ++i) {
    const Dims& d = pv[i].d;
    const int S = (int)in[i].n_samples, c = d.cplx ? 1 : 0;
    int items[kGroupLists];
    group_items(d, S, items);
    for (int q = 0; q < kGroupLists; ++q) lists_b[q].add(i, items[q]);
    maxN[c] = d.N > maxN[c] ? d.N : maxN[c];
    T_max = in[i].n_keep > T_max ? (int)in[i].n_keep : T_max;
  }
  ListBuild* lists[kGroupLists];
  for (int q = 0; q < kGroupLists; ++q) lists[q] = &lists_b[q];
  size_t tab = rup((size_t)n * sizeof(GInst), 256);
  size_t list_off[kGroupLists];
  for (int k = 0; k < kGroupLists; ++k) {
    list_off[k] = tab;
    tab += rup((lists[k]->ids.size() + lists[k]->pre.size()) * sizeof(int), 256);
  }
  const size_t stat_off = tab;  // pinned only: per-instance counters copied back
  const size_t pinned_bytes = stat_off + (size_t)n * 32;
  std::vector<size_t> w_off(n);
  size_t total = tab;
  for (int i = 0; i < n; ++i) {
    w_off[i] = total;
    total += rup(carve(pv[i].d, nullptr, (int)rup(in[i].n_samples, SAMPLE_PAD), nullptr), 256);
  }

  std::lock_guard<std::mutex> guard(g_stage.mu);
  for (size_t k = 0; k < g_stage.dead.size();) {  // release finished graphs
    if (hipEventQuery(g_stage.dead[k].done) == hipSuccess) {
      (void)hipGraphExecDestroy(g_stage.dead[k].exec);
      (void)hipGraphDestroy(g_stage.dead[k].graph);
      (void)hipEventDestroy(g_stage.dead[k].done);
      g_stage.dead.erase(g_stage.dead.begin() + k);
    } else {
      ++k;
    }
  }
  if (g_stage.device >= 0) (void)hipEventSynchronize(g_stage.uploaded);
  if (pinned_bytes > g_stage.cap) {
    if (g_stage.host) (void)hipHostFree(g_stage.host);
    g_stage.host = nullptr;
    g_stage.cap = 0;
    if (hipHostMalloc(&g_stage.host, pinned_bytes, 0) != hipSuccess)
      return (ffs_status)set_error(FFS_ERR_OUT_OF_MEMORY, "pinned staging allocation failed");
    g_stage.cap = pinned_bytes;
  }
  if (g_stage.device != dev) {  // first call (or another device): own stream and events
    if (g_stage.device >= 0)
      return (ffs_status)set_error(FFS_ERR_UNSUPPORTED, "grouped runs use one device per process");
    if (hipEventCreateWithFlags(&g_stage.uploaded, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&g_stage.ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&g_stage.ev_join, hipEventDisableTiming) != hipSuccess ||
        hipStreamCreateWithFlags(&g_stage.st, hipStreamNonBlocking) != hipSuccess)
      return (ffs_status)set_error(FFS_ERR_HIP, "stream or event creation failed");
    g_stage.device = dev;
  }
  hipStream_t user = static_cast<hipStream_t>(stream), st = g_stage.st;
  (void)hipEventRecord(g_stage.ev_fork, user);
  (void)hipStreamWaitEvent(st, g_stage.ev_fork, 0);
  char* mem = nullptr;
  if (hipMallocAsync((void**)&mem, total, st) != hipSuccess)
    return (ffs_status)set_error(FFS_ERR_OUT_OF_MEMORY, "group working memory");

  // ---- instance table and lists (host side, then one upload) -------------
  char* hst = static_cast<char*>(g_stage.host);
  GInst* hi = reinterpret_cast<GInst*>(hst);
  std::vector<Work> works(n);
  for (int i = 0; i < n; ++i) {
    const Dims& d = pv[i].d;
    const ffs_instance& q = in[i];
    const int S = (int)q.n_samples;
    carve(d, mem + w_off[i], (int)rup(S, SAMPLE_PAD), &works[i]);
    hi[i] = make_ginst(pv[i], works[i], S, (int)q.n_keep, q.seed, q.first_sample);
  }
  GList gl[kGroupLists];
  for (int k = 0; k < kGroupLists; ++k) {
    int* h = reinterpret_cast<int*>(hst + list_off[k]);
    const size_t ni = lists[k]->ids.size();
    memcpy(h, lists[k]->ids.data(), ni * sizeof(int));
    memcpy(h + ni, lists[k]->pre.data(), lists[k]->pre.size() * sizeof(int));
    int* dv = reinterpret_cast<int*>(mem + list_off[k]);
    gl[k].ids = dv;
    gl[k].pre = dv + ni;
    gl[k].n = (int)ni;
    gl[k].total = lists[k]->pre.back();
  }
  GInst* inst = reinterpret_cast<GInst*>(mem);
  hipError_t e = hipMemcpyAsync(mem, hst, stat_off, hipMemcpyHostToDevice, st);
  (void)hipEventRecord(g_stage.uploaded, st);

  // ---- first step of every instance, then the ticks ------------------------
  for (int i = 0; i < n && e == hipSuccess; ++i)
    start_instance(pv[i], works[i], (int)in[i].n_samples, (int)in[i].n_keep, in[i].seed,
                   in[i].first_sample, st);
  auto tick = [&]() { launch_tick(inst, gl, maxN, n, st); };
  ffs_status status = FFS_OK;
  if (e != hipSuccess) {
    status = (ffs_status)set_error(FFS_ERR_HIP, "table upload failed");
  } else if (flags & FFS_GROUP_GRAPH) {
    const int G = T_max < 16 ? T_max : 16;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      for (int g = 0; g < G; ++g) tick();
      e = hipStreamEndCapture(st, &graph);
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e == hipSuccess) {
      for (int r = 0; r < (T_max + G - 1) / G && e == hipSuccess; ++r) e = hipGraphLaunch(exec, st);
      hipEvent_t done = nullptr;
      (void)hipEventCreateWithFlags(&done, hipEventDisableTiming);
      (void)hipEventRecord(done, st);
      g_stage.dead.push_back({exec, graph, done});
    } else if (graph) {
      (void)hipGraphDestroy(graph);
    }
    if (e != hipSuccess) status = (ffs_status)set_error(FFS_ERR_HIP, hipGetErrorString(e));
  } else {
    for (int t = 0; t < T_max; ++t) tick();
  }
  for (int i = 0; i < n && status == FFS_OK; ++i) {
    launch_copy_out(pv[i].d, works[i], (int)in[i].n_samples, (int)in[i].n_keep, in[i].x_dev,
                    in[i].logdet_dev, st);
    if (stats) {
      char* dst = hst + stat_off + (size_t)i * 32;
      (void)hipMemcpyAsync(dst, works[i].counters, 16, hipMemcpyDeviceToHost, st);
      (void)hipMemcpyAsync(dst + 16, works[i].ctl, 8, hipMemcpyDeviceToHost, st);
    }
  }
  (void)hipFreeAsync(mem, st);
  if ((e = hipGetLastError()) != hipSuccess && status == FFS_OK)
    status = (ffs_status)set_error(FFS_ERR_HIP, hipGetErrorString(e));
  (void)hipEventRecord(g_stage.ev_join, st);
  (void)hipStreamWaitEvent(user, g_stage.ev_join, 0);
  if (stats) {
    (void)hipStreamSynchronize(st);
    for (int i = 0; i < n; ++i) {
      const char* src = hst + stat_off + (size_t)i * 32;
      unsigned long long c[2];
      int32_t ctl[2];
      memcpy(c, src, 16);
      memcpy(ctl, src + 16, 8);
      stats[i].draws = in[i].n_samples * in[i].n_keep;
      stats[i].flagged = (int64_t)c[0];
      stats[i].changed = (int64_t)c[1];
      stats[i].device_status = (ctl[1] & DEV_NUMERICAL) ? FFS_ERR_NUMERICAL : FFS_OK;
      stats[i].reserved = 0;
    }
  }
  return status;
}
