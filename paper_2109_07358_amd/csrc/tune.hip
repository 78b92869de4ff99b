// Tile autotuner of the float32 contraction.
//
// The contraction has tile variants that differ only in how sites and
// samples are tiled (never in the order of the K reduction), so any of them
// gives bit-identical results.  ffs_autotune times every variant allowed
// for a plan on the launch shapes a call of n samples uses (two halves when
// the plan overlaps them) and records the fastest per shape (L_pad, K,
// samples per launch, complex); launches consult the table and fall back to
// the 128 x 128 tile.  With FFS_TUNE_FILE set, the table is read from that
// file on first use and the file is rewritten after each tuning: a small
// JSON document, one entry per line.
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/ffs.h"
#include "ffs_internal.h"

namespace ffsk {
namespace {

struct Key {
  int L_pad, Kg, S, cplx;
  bool operator<(const Key& o) const {
    if (L_pad != o.L_pad) return L_pad < o.L_pad;
    if (Kg != o.Kg) return Kg < o.Kg;
    if (S != o.S) return S < o.S;
    return cplx < o.cplx;
  }
};

std::mutex g_mu;
std::map<Key, int> g_table;
bool g_loaded = false;

int variant_of(int sites, int cols, int kc) {
  for (int v = 0; v < kNumTilesDecl; ++v)
    if (kTiles[v].sites == sites && kTiles[v].cols == cols && kTiles[v].kc == kc) return v;
  return -1;
}

// "SITESxCOLS" for a 32-wide K chunk, "SITESxCOLSkKC" otherwise.
void tile_name(int v, char* out, size_t n) {
  if (kTiles[v].kc == 32)
    snprintf(out, n, "%dx%d", kTiles[v].sites, kTiles[v].cols);
  else
    snprintf(out, n, "%dx%dk%d", kTiles[v].sites, kTiles[v].cols, kTiles[v].kc);
}

int parse_tile(const char* s) {
  int ts = 0, tc = 0, kc = 32;
  const int n = sscanf(s, "%dx%dk%d", &ts, &tc, &kc);
  if (n < 2) return -1;
  return variant_of(ts, tc, n == 3 ? kc : 32);
}

void load_locked() {
  if (g_loaded) return;
  g_loaded = true;
  const char* path = getenv("FFS_TUNE_FILE");
  if (!path || !*path) return;
  FILE* f = fopen(path, "r");
  if (!f) return;
  char line[512];
  while (fgets(line, sizeof line, f)) {
    Key k;
    char name[32] = {0};
    if (sscanf(line, " {\"L_pad\": %d, \"K\": %d, \"S\": %d, \"complex\": %d, \"tile\": \"%31[0-9xk]\"",
               &k.L_pad, &k.Kg, &k.S, &k.cplx, name) == 5) {
      const int v = parse_tile(name);
      if (v >= 0) g_table[k] = v;
    }
  }
  fclose(f);
}

void save_locked() {
  const char* path = getenv("FFS_TUNE_FILE");
  if (!path || !*path) return;
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = fopen(tmp.c_str(), "w");
  if (!f) return;
  fprintf(f, "{\"ffs_tile_choices\": [\n");
  size_t i = 0;
  for (const auto& kv : g_table) {
    char name[32];
    tile_name(kv.second, name, sizeof name);
    fprintf(f, "  {\"L_pad\": %d, \"K\": %d, \"S\": %d, \"complex\": %d, \"tile\": \"%s\"}%s\n",
            kv.first.L_pad, kv.first.Kg, kv.first.S, kv.first.cplx, name,
            ++i < g_table.size() ? "," : "");
  }
  fprintf(f, "]}\n");
  fclose(f);
  rename(tmp.c_str(), path);
}

inline int rup(int v, int m) { return (v + m - 1) / m * m; }

}  // namespace

int tile_choice(const Dims& d, int s_round) {
  {
    std::lock_guard<std::mutex> g(g_mu);
    load_locked();
    const auto it = g_table.find(Key{d.L_pad, d.Kg, s_round, d.cplx});
    if (it != g_table.end() && tile_allowed(d, it->second)) return it->second;
  }
  // untuned: the 16-wide K chunk, which measured faster than the 32-wide one
  // for every tile and shape tried; real: 64 x 64 (best or within 1% of the
  // best alone and clearly best beside the other half-batch's factor work);
  // complex (128 GEMM columns only): 128 x 128 unless it would leave the
  // 256 CUs short of work
  if (!d.cplx) return 7;
  const int wg = (d.L_pad / 128) * (s_round / 64);
  return wg >= 256 ? 4 : 5;
}

}  // namespace ffsk

using namespace ffsk;

namespace {
// Samples per contraction launch (rounded to SAMPLE_PAD) of a call of n.
std::vector<int> launch_shapes(const PlanView& pv, int64_t n) {
  const int chunk = (int)(n < pv.max_batch ? n : pv.max_batch);
  std::vector<int> shapes;
  if (pv.overlap && chunk >= 2 * SAMPLE_PAD) {
    int a = rup((chunk + 1) / 2, SAMPLE_PAD);
    a = a < chunk ? a : chunk;
    shapes.push_back(rup(a, SAMPLE_PAD));
    if (rup(chunk - a, SAMPLE_PAD) != shapes[0]) shapes.push_back(rup(chunk - a, SAMPLE_PAD));
  } else {
    shapes.push_back(rup(chunk, SAMPLE_PAD));
  }
  return shapes;
}
}  // namespace

extern "C" ffs_status ffs_set_tile(ffs_plan_t p, int64_t n_samples, int32_t sites,
                                   int32_t cols, int32_t kchunk) {
  if (!p || n_samples < 1) return (ffs_status)set_error(FFS_ERR_INVALID_ARG, "bad plan or n_samples");
  const PlanView pv = plan_view(p);
  const int v = variant_of(sites, cols, kchunk == 0 ? 32 : kchunk);
  if (v < 0 || !tile_allowed(pv.d, v))
    return (ffs_status)set_error(FFS_ERR_INVALID_ARG, "no such tile for this plan");
  std::lock_guard<std::mutex> lk(g_mu);
  load_locked();
  for (int S : launch_shapes(pv, n_samples)) g_table[Key{pv.d.L_pad, pv.d.Kg, S, pv.d.cplx}] = v;
  return FFS_OK;
}

// Pipeline tuning: every tile is tried on a short sampling call (the first
// steps of n samples) with the rest of the step running alongside, and the
// fastest whole call wins.
static ffs_status tune_pipeline(ffs_plan_t p, const PlanView& pv, int64_t n,
                                char* choice_out) {
  const int keep = pv.d.N < 32 ? pv.d.N : 32;
  int32_t* x = nullptr;
  if (hipMalloc(&x, (size_t)n * keep * 4) != hipSuccess)
    return (ffs_status)set_error(FFS_ERR_OUT_OF_MEMORY, "tuning buffers");
  hipEvent_t e0 = nullptr, e1 = nullptr;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  const std::vector<int> shapes = launch_shapes(pv, n);
  int best = 0;
  float best_ms = 1e30f;
  ffs_status st = FFS_OK;
  for (int v = 0; v < kNumTilesDecl && st == FFS_OK; ++v) {
    if (!tile_allowed(pv.d, v)) continue;
    {
      std::lock_guard<std::mutex> lk(g_mu);
      load_locked();
      for (int S : shapes) g_table[Key{pv.d.L_pad, pv.d.Kg, S, pv.d.cplx}] = v;
    }
    if ((st = ffs_marginal(p, keep, 0x7E57, 0, n, x, nullptr)) != FFS_OK) break;  // warm-up
    (void)hipEventRecord(e0, nullptr);
    for (int r = 0; r < 2 && st == FFS_OK; ++r) st = ffs_marginal(p, keep, 0x7E57, 0, n, x, nullptr);
    (void)hipEventRecord(e1, nullptr);
    if (hipEventSynchronize(e1) != hipSuccess) st = (ffs_status)set_error(FFS_ERR_HIP, "tuning");
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (ms < best_ms) {
      best_ms = ms;
      best = v;
    }
  }
  {
    std::lock_guard<std::mutex> lk(g_mu);
    for (int S : shapes) g_table[Key{pv.d.L_pad, pv.d.Kg, S, pv.d.cplx}] = best;
    if (st == FFS_OK) save_locked();
  }
  if (choice_out) tile_name(best, choice_out, 32);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(x);
  return st;
}

extern "C" ffs_status ffs_autotune(ffs_plan_t p, int64_t n_samples, int32_t flags,
                                   char* choice_out) {
  if (flags & ~FFS_TUNE_PIPELINE) return (ffs_status)set_error(FFS_ERR_INVALID_ARG, "unknown flags");
  if (!p || n_samples < 1) return (ffs_status)set_error(FFS_ERR_INVALID_ARG, "bad plan or n_samples");
  if (plan_path(p) != FFS_PATH_BATCHED)
    return (ffs_status)set_error(FFS_ERR_INVALID_ARG, "tuning applies to the batched path");
  const PlanView pv = plan_view(p);
  const Dims& d = pv.d;
  if (d.bf16) {  // a single split-bfloat16 tile
    if (choice_out) snprintf(choice_out, 32, "128x128");
    return FFS_OK;
  }
  if (flags & FFS_TUNE_PIPELINE) return tune_pipeline(p, pv, n_samples, choice_out);
  const std::vector<int> shapes = launch_shapes(pv, n_samples);
  const int s_max = shapes[0] > shapes.back() ? shapes[0] : shapes.back();
  Work w;
  const size_t bytes = carve(d, nullptr, s_max, nullptr);
  void* mem = nullptr;
  if (hipMalloc(&mem, bytes) != hipSuccess)
    return (ffs_status)set_error(FFS_ERR_OUT_OF_MEMORY, "tuning buffers");
  carve(d, static_cast<char*>(mem), s_max, &w);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ffs_status status = FFS_OK;
  if (hipMemset(w.gam, 0, (size_t)s_max * d.Kg * 4) != hipSuccess ||
      hipMemset(w.occ, 0, (size_t)s_max * (d.L_pad / 32) * 4) != hipSuccess ||
      hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    status = (ffs_status)set_error(FFS_ERR_HIP, "tuning setup");
  const WArgs g = make_wargs(d, w, pv.ubulk);
  int first_choice = 0;
  for (size_t si = 0; si < shapes.size() && status == FFS_OK; ++si) {
    const int S = shapes[si];
    int best = 0;
    float best_ms = 1e30f;
    for (int v = 0; v < kNumTilesDecl; ++v) {
      if (!tile_allowed(d, v)) continue;
      for (int r = 0; r < 2; ++r) launch_weights_variant(d, g, S, v, nullptr);
      (void)hipEventRecord(e0, nullptr);
      for (int r = 0; r < 5; ++r) launch_weights_variant(d, g, S, v, nullptr);
      (void)hipEventRecord(e1, nullptr);
      if (hipEventSynchronize(e1) != hipSuccess) {
        status = (ffs_status)set_error(FFS_ERR_HIP, "tuning launch failed");
        break;
      }
      float ms = 0.0f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (ms < best_ms) {
        best_ms = ms;
        best = v;
      }
    }
    if (si == 0) first_choice = best;
    std::lock_guard<std::mutex> lk(g_mu);
    load_locked();
    g_table[Key{d.L_pad, d.Kg, S, d.cplx}] = best;
  }
  if (status == FFS_OK) {
    std::lock_guard<std::mutex> lk(g_mu);
    save_locked();
  }
  if (choice_out) tile_name(first_choice, choice_out, 32);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(mem);
  return status;
}
