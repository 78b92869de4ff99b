// Host side of the C ABI: plan creation (validation, U layouts on the
// device), per-stream working memory, the step loop of the batched path and
// the per-sample launches of the plain path.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <complex>
#include <map>
#include <atomic>
#include <mutex>
#include <random>
#include <string>
#include <vector>

#include "../../include/ffs.h"
#include "ffs_internal.h"

using namespace ffsk;

namespace {

thread_local std::string g_err;

ffs_status fail(ffs_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIP_OK(call)                                                        \
  do {                                                                      \
    hipError_t e_ = (call);                                                 \
    if (e_ != hipSuccess)                                                   \
      return fail(e_ == hipErrorOutOfMemory ? FFS_ERR_OUT_OF_MEMORY          \
                                            : FFS_ERR_HIP,                  \
                  "%s: %s", #call, hipGetErrorString(e_));                  \
  } while (0)

inline int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

// bfloat16 bits of a finite float, rounded to nearest even, and back.
inline uint16_t bf16_bits(float x) {
  uint32_t u;
  memcpy(&u, &x, 4);
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
inline float bf16_value(uint16_t h) {
  const uint32_t u = (uint32_t)h << 16;
  float x;
  memcpy(&x, &u, 4);
  return x;
}

// Working memory of one stream.  Batches of at least 2*SAMPLE_PAD samples
// are split in two halves, each with its own buffers, the second half
// running on an internal stream: the latency-bound float64 factor update of
// one half then overlaps the matrix-core contraction of the other.
struct Slot {
  Work w;   // first half (or the whole batch)
  Work w2;  // second half
  int S_cap = 0;   // samples per half-buffer
  std::vector<void*> allocs;
  void* plain_scratch = nullptr;
  hipStream_t s2 = nullptr;
  hipEvent_t ev_fork = nullptr, ev_phase = nullptr, ev_join = nullptr;
  // deferred resolution: the host copy of the listed counts, the replay
  // batch's memory, and whether the slot's last call ran a replay (read by
  // ffs_check)
  int32_t* listed_host = nullptr;  // pinned [2]
  Slot* replay = nullptr;
  bool replayed = false;
};

}  // namespace

struct ffs_plan_s {
  Dims d;
  ffs_options opt;
  double g_fixed = 0.0, g_coef = 0.0;  // guard: fixed relative margin, adaptive factor
  int device = 0;
  void* u64 = nullptr;    // [L][N]
  void* u64t = nullptr;   // [N][L_pad]
  void* ubulk = nullptr;  // [Kg rows][L_pad] float32
  void* ubf = nullptr;    // split-bfloat16 heads then tails, [Kg/32][L_pad][32] each
  int32_t* anchor = nullptr;  // [N] first row of largest |U[., c]|^2 (Metropolis start)
  // ffs_sample / ffs_marginal resolve flagged draws at the call's end; under
  // AUTO a call that needed a replay turns it off for the plan's later calls
  // (a replay costs a per-step run of its samples, more than the launches
  // deferral saves), which changes their speed, never their results
  std::atomic<bool> deferred{false};
  bool deferred_auto = false;
  std::mutex mu;
  std::map<hipStream_t, Slot*> slots;
  std::map<hipStream_t, Slot*> subset_slots;  // column-subset calls (sized by k, S)
  std::map<hipStream_t, int> subset_kcap;
  // ffs_sample_dpp: size groups run round-robin on the caller's stream and
  // these (created on first use, default priority); one call at a time per
  // plan (dpp_mu), since the groups' subset runs fill per-stream host state
  static constexpr int kDppStreams = 3;
  hipStream_t dpp_st[kDppStreams] = {};
  hipEvent_t dpp_fork = nullptr;
  hipEvent_t dpp_join[kDppStreams] = {};
  std::mutex dpp_mu;
  Slot* last_slot = nullptr;
  hipEvent_t last_event = nullptr;
  int64_t last_draws = 0;
  // measurement hook (ffs_set_timing): event pairs per launch, by class;
  // bit c of timing = record class c
  uint32_t timing = 0;
  // ffs_set_timing_stride: one launch in `timing_stride` of each timed
  // class is bracketed (counted per class)
  int timing_stride = 1;
  int64_t timing_seen[FFS_K_COUNT] = {};
  struct Rec {
    int cls;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  // contraction launches are timed on the device's steady clock: a pair
  // (earliest workgroup start, latest workgroup end) per launch
  unsigned long long* kstamp = nullptr;
  int kstamp_cap = 0, kstamp_n = 0;
  double wall_khz = 0.0;
};

namespace {

// Brackets one launch with an event pair on `st` when timing is enabled.
struct Timed {
  ffs_plan_s* p;
  hipStream_t st;
  int cls;
  hipEvent_t a = nullptr, b = nullptr;
  hipEvent_t take() {
    if (!p->pool.empty()) {
      hipEvent_t e = p->pool.back();
      p->pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
  }
  // stamped = true: the events are handed to the launch (a, b), which has
  // the dispatch stamp them with the kernel's own start and end, instead of
  // being recorded on the stream around it (that interval also holds the
  // wait for CUs that the other half-batch's kernels occupy).
  bool stamped = false;
  Timed(ffs_plan_s* p_, hipStream_t s_, int c_, bool on = true, bool stamped_ = false)
      : p(p_), st(s_), cls(c_), stamped(stamped_) {
    if (!on || !((p->timing >> c_) & 1u)) return;
    if (p->timing_seen[c_]++ % p->timing_stride != 0) return;
    a = take();
    b = take();
    if (!stamped) (void)hipEventRecord(a, st);
  }
  ~Timed() {
    if (!a) return;
    if (!stamped) (void)hipEventRecord(b, st);
    p->recs.push_back({cls, a, b});
  }
};

// A device stamp pair for one contraction launch when its class is timed
// (nullptr otherwise, or when the stamp buffer is full); read by
// ffs_kernel_spans, next to the launch's event pair.
unsigned long long* take_stamp(ffs_plan_s* p, bool on) {
  if (!on || !((p->timing >> FFS_K_WEIGHTS) & 1u) || !p->kstamp || p->kstamp_n >= p->kstamp_cap)
    return nullptr;
  return p->kstamp + 2 * (size_t)(p->kstamp_n++);
}

// Stamp pairs start as (max, 0) so the launch's min / max updates land.
hipError_t reset_stamps(ffs_plan_s* p, int n) {
  if (!p->kstamp || n <= 0) return hipSuccess;
  std::vector<unsigned long long> h(2 * (size_t)n);
  for (int i = 0; i < n; ++i) {
    h[2 * (size_t)i] = ~0ull;
    h[2 * (size_t)i + 1] = 0ull;
  }
  return hipMemcpy(p->kstamp, h.data(), h.size() * 8, hipMemcpyHostToDevice);
}

// Allocates the stamp buffer the first time the contraction class is timed.
ffs_status ensure_stamps(ffs_plan_s* p) {
  if (p->kstamp || !((p->timing >> FFS_K_WEIGHTS) & 1u)) return FFS_OK;
  int khz = 0;
  HIP_OK(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, p->device));
  if (khz <= 0) return FFS_OK;  // no steady clock: the contraction keeps its events
  const int cap = 1 << 16;
  HIP_OK(hipMalloc(&p->kstamp, (size_t)cap * 16));
  p->kstamp_cap = cap;
  p->kstamp_n = 0;
  p->wall_khz = (double)khz;
  HIP_OK(reset_stamps(p, cap));
  return FFS_OK;
}

}  // namespace

namespace {

void free_slot(Slot* s) {
  for (void* p : s->allocs) (void)hipFree(p);
  s->allocs.clear();
  s->S_cap = 0;
  s->w = Work();
  s->w2 = Work();
  s->plain_scratch = nullptr;
}

// Record slots of deferred resolution per sample of a batch (one pool per
// batch): max(2, N/64).  With the default float32 guard a call flags about
// one draw in 16k at L = 4096, N = 256 and 0.55% of draws (2.8 per sample)
// at L = 16384, N = 512 complex, well inside the pool; a sample whose
// record finds no slot is replayed, so the pool size never changes results.
inline int records_per_sample(int N) { return N / 64 > 2 ? N / 64 : 2; }

// Lays the buffers of one batch of S_pad samples out from `base` (256-byte
// aligned pieces) and returns the total size; with base == nullptr only the
// size is computed.
size_t carve_work(const Dims& d, char* base, int S_pad, Work* w, bool rec = false) {
  const size_t es = d.cplx ? 16 : 8;
  const size_t nblk = d.L_pad / 32;
  size_t off = 0;
  auto take = [&](size_t bytes) -> void* {
    void* r = base ? base + off : nullptr;
    off += round_up((int64_t)(bytes < 256 ? 256 : bytes), 256);
    return r;
  };
  Work t;
  t.perm = (int32_t*)take((size_t)S_pad * d.N * 4);
  t.xs = (int32_t*)take((size_t)S_pad * d.N * 4);
  t.F = take((size_t)S_pad * factor_state_bytes(d));
  t.beta = take((size_t)S_pad * d.N * es);
  t.logdet = (double*)take((size_t)S_pad * 8);
  t.gam = take((size_t)S_pad * d.Kg * 4);
  t.occ = (uint32_t*)take((size_t)S_pad * nblk * 4);
  t.wh = take((size_t)S_pad * d.L_pad * 4);
  t.bsum = (double*)take(nblk * S_pad * 8);
  t.ctl = (int32_t*)take(256);
  t.flag_list = (int32_t*)take((size_t)S_pad * 4);
  t.counters = (unsigned long long*)take(256);
  t.wr = (double*)take((size_t)S_pad * d.L_pad * 8);
  t.cs = (double*)take((size_t)S_pad * (d.L_pad / RCHUNK) * 8);
  t.g64 = take((size_t)S_pad * d.Np * es);
  t.forced = (int32_t*)take((size_t)d.N * 4);
  t.cmap_buf = (int32_t*)take((size_t)S_pad * d.N * 4);
  t.fslot = (int32_t*)take((size_t)S_pad * 4);
  t.rec_ctl = (int32_t*)take(256);
  t.div = (int32_t*)take((size_t)S_pad * 4);
  t.rep_row = (int32_t*)take((size_t)S_pad * 4);
  t.rep_sid = (uint64_t*)take((size_t)S_pad * 8);
  if (rec) {  // records of a deferred call
    t.rec_cap = records_per_sample(d.N) * S_pad;
    t.rec_meta = (int32_t*)take((size_t)t.rec_cap * 16);
    t.rec_g = take((size_t)t.rec_cap * d.Np * es);
    t.rec_occ = (uint32_t*)take((size_t)t.rec_cap * nblk * 4);
  }
  t.S_pad = S_pad;
  if (w) *w = t;
  return off;
}

size_t slot_bytes(const Dims& d, int S_pad, bool rec = false) {
  return carve_work(d, nullptr, S_pad, nullptr, rec);
}

ffs_status alloc_work(ffs_plan_s* p, Slot* s, Work& w, int S_pad, bool rec = false) {
  const Dims& d = p->d;
  void* base = nullptr;
  const size_t bytes = carve_work(d, nullptr, S_pad, nullptr, rec);
  hipError_t e = hipMalloc(&base, bytes);
  if (e != hipSuccess) {
    free_slot(s);
    return fail(FFS_ERR_OUT_OF_MEMORY, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
  }
  s->allocs.push_back(base);
  carve_work(d, static_cast<char*>(base), S_pad, &w, rec);
  HIP_OK(hipMemset(w.gam, 0, (size_t)S_pad * d.Kg * 4));
  HIP_OK(hipMemset(w.ctl, 0, 256));
  HIP_OK(hipMemset(w.counters, 0, 256));
  w.S_pad = S_pad;
  return FFS_OK;
}

// Batches of at least 2*SAMPLE_PAD samples run as two halves.
inline bool split_batch(int S) { return S >= 2 * SAMPLE_PAD; }
inline int first_half(int S) {
  const int h = (int)round_up((S + 1) / 2, SAMPLE_PAD);
  return h < S ? h : S;
}

// rec: the buffers also hold the records of deferred resolution.
ffs_status ensure_slot(ffs_plan_s* p, Slot* s, int S, bool rec = false) {
  const bool split = p->opt.overlap && split_batch(S);
  const int per = (int)round_up(split ? first_half(S) : S, SAMPLE_PAD);
  if (per <= s->S_cap && (!split || s->w2.S_pad > 0) && (!rec || s->w.rec_cap > 0))
    return FFS_OK;
  const int cap = per > s->S_cap ? per : s->S_cap;
  const bool two = split || s->w2.S_pad > 0;
  free_slot(s);
  ffs_status st;
  if ((st = alloc_work(p, s, s->w, cap, rec)) != FFS_OK) return st;
  if (two && (st = alloc_work(p, s, s->w2, cap, rec)) != FFS_OK) return st;
  s->S_cap = cap;
  return FFS_OK;
}

Slot* get_slot(ffs_plan_s* p, hipStream_t st) {
  std::lock_guard<std::mutex> g(p->mu);
  auto it = p->slots.find(st);
  if (it != p->slots.end()) return it->second;
  Slot* s = new Slot();
  p->slots[st] = s;
  return s;
}

// Max |U^H U - 1|: exact for small problems, randomised probes otherwise.
inline double conj_(double v) { return v; }
inline std::complex<double> conj_(std::complex<double> v) { return std::conj(v); }

template <typename Cplx>
double ortho_error(const Cplx* U, int64_t L, int64_t N, int64_t ldu,
                   bool* randomised) {
  const double lim = (double)(1 << 28);
  if ((double)L * N * N <= lim) {
    *randomised = false;
    double err = 0.0;
    std::vector<Cplx> G((size_t)N * N, Cplx(0));
    for (int64_t i = 0; i < L; ++i) {
      const Cplx* r = U + i * ldu;
      for (int64_t a = 0; a < N; ++a) {
        const Cplx ca = conj_(r[a]);
        Cplx* g = &G[(size_t)a * N];
        for (int64_t b = 0; b < N; ++b) g[b] += ca * r[b];
      }
    }
    for (int64_t a = 0; a < N; ++a)
      for (int64_t b = 0; b < N; ++b) {
        const Cplx e = G[(size_t)a * N + b] - (a == b ? Cplx(1) : Cplx(0));
        err = fmax(err, std::abs(e));
      }
    return err;
  }
  *randomised = true;
  std::mt19937_64 gen(12345);
  std::normal_distribution<double> nd;
  double worst = 0.0;
  std::vector<Cplx> z(N), y(L), v(N);
  for (int probe = 0; probe < 4; ++probe) {
    double zn = 0.0;
    for (auto& e : z) {
      e = Cplx(nd(gen));
      zn += std::norm(e);
    }
    zn = sqrt(zn);
    for (int64_t i = 0; i < L; ++i) {
      Cplx acc(0);
      for (int64_t b = 0; b < N; ++b) acc += U[i * ldu + b] * z[b];
      y[i] = acc;
    }
    std::fill(v.begin(), v.end(), Cplx(0));
    for (int64_t i = 0; i < L; ++i)
      for (int64_t a = 0; a < N; ++a) v[a] += conj_(U[i * ldu + a]) * y[i];
    for (int64_t a = 0; a < N; ++a) worst = fmax(worst, std::abs(v[a] - z[a]) / zn);
  }
  return worst;
}

}  // namespace

extern "C" {

void ffs_default_options(ffs_options* o) {
  if (!o) return;
  o->bulk = FFS_BULK_FP32;
  o->path = FFS_PATH_BATCHED;
  o->ortho_tol = 1e-10;
  o->guard_delta = -1.0;
  o->max_batch = 4096;
  o->hbm_budget = 0;
  o->overlap = 1;
  o->resolve = FFS_RESOLVE_AUTO;
  o->guard_scale = -1.0;
}

const char* ffs_last_error(void) { return g_err.c_str(); }

void ffs_philox_words(uint64_t seed, uint64_t sample, uint32_t step,
                      uint32_t* out) {
  if (!out) return;
  const Words w = philox_block(seed, sample, step);
  out[0] = w.w0;
  out[1] = w.w1;
  out[2] = w.w2;
  out[3] = w.w3;
}

ffs_status ffs_plan(ffs_plan_t* out, const void* U_host, int64_t L, int64_t N,
                    int64_t ldu, int32_t dtype, const ffs_options* opt) {
  if (!out) return fail(FFS_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!U_host) return fail(FFS_ERR_INVALID_ARG, "U_host is NULL");
  if (dtype != FFS_REAL64 && dtype != FFS_COMPLEX128)
    return fail(FFS_ERR_INVALID_ARG, "unknown dtype %d", (int)dtype);
  if (N < 1 || L < N) return fail(FFS_ERR_INVALID_ARG, "need 1 <= N <= L (L=%lld N=%lld)", (long long)L, (long long)N);
  if (ldu < N) return fail(FFS_ERR_INVALID_ARG, "ldu < N");
  if (N > 1024) return fail(FFS_ERR_UNSUPPORTED, "N=%lld above 1024", (long long)N);
  if (L > 65536) return fail(FFS_ERR_UNSUPPORTED, "L=%lld above 65536", (long long)L);
  ffs_options o;
  ffs_default_options(&o);
  if (opt) o = *opt;
  if (o.bulk != FFS_BULK_FP32 && o.bulk != FFS_BULK_FP64 && o.bulk != FFS_BULK_SPLIT_BF16)
    return fail(FFS_ERR_INVALID_ARG, "unknown bulk mode %d", (int)o.bulk);
  if (o.path != FFS_PATH_BATCHED && o.path != FFS_PATH_PLAIN)
    return fail(FFS_ERR_INVALID_ARG, "unknown path %d", (int)o.path);
  if (o.path == FFS_PATH_BATCHED && o.bulk == FFS_BULK_FP64)
    return fail(FFS_ERR_UNSUPPORTED, "float64 bulk is available on the plain path only");
  if (o.path == FFS_PATH_PLAIN && o.bulk == FFS_BULK_SPLIT_BF16)
    return fail(FFS_ERR_UNSUPPORTED, "split-bfloat16 bulk is available on the batched path only");
  if (!(o.ortho_tol > 0.0) || isnan(o.guard_delta) || isnan(o.guard_scale) ||
      !isfinite(o.guard_scale) || o.max_batch < 1 ||
      (o.overlap != 0 && o.overlap != 1) || o.resolve < FFS_RESOLVE_AUTO ||
      o.resolve > FFS_RESOLVE_DEFERRED)
    return fail(FFS_ERR_INVALID_ARG, "bad options");
  if (o.resolve == FFS_RESOLVE_DEFERRED && o.path != FFS_PATH_BATCHED)
    return fail(FFS_ERR_UNSUPPORTED, "deferred resolution is a batched-path mode");
  // Guard threshold of a draw: max(delta * T, coef * sqrt(sum_b B_b^2)).  The
  // adaptive term's unit is the float32 CDF error scale 2^-24 sqrt(K), K the
  // contraction's length (N real; 2N complex, a complex weight's count of
  // real products in the real embedding, kept for the Gauss form);
  // the default factor is 2 for float32 (>= 10x the largest CDF error
  // measured in that unit) and 32 for split-bfloat16 (>= 9x).  A fixed
  // guard_delta alone (guard_scale left at -1) turns the adaptive term off.
  const double unit = 0x1.0p-24 * sqrt((double)(dtype == FFS_COMPLEX128 ? 2 * N : N));
  const double def_scale = o.bulk == FFS_BULK_SPLIT_BF16 ? 32.0
                           : o.bulk == FFS_BULK_FP32     ? 2.0
                                                         : 0.0;
  const double g_fixed = o.guard_delta >= 0.0 ? o.guard_delta : 0.0;
  const double g_coef = o.guard_scale >= 0.0 ? o.guard_scale * unit
                        : o.guard_delta >= 0.0 ? 0.0
                                               : def_scale * unit;
  const bool cplx = dtype == FFS_COMPLEX128;
  const double* H = static_cast<const double*>(U_host);
  for (int64_t i = 0; i < L; ++i)
    for (int64_t j = 0; j < N * (cplx ? 2 : 1); ++j)
      if (!isfinite(H[i * ldu * (cplx ? 2 : 1) + j]))
        return fail(FFS_ERR_NUMERICAL, "non-finite entry at row %lld", (long long)i);
  bool randomised = false;
  const double oerr =
      cplx ? ortho_error(static_cast<const std::complex<double>*>(U_host), L, N, ldu, &randomised)
           : ortho_error(static_cast<const double*>(U_host), L, N, ldu, &randomised);
  if (!(oerr <= o.ortho_tol))
    return fail(FFS_ERR_NOT_ORTHONORMAL, "max |U^H U - 1| = %.3e > %.3e (%s check)",
                oerr, o.ortho_tol, randomised ? "randomised" : "exact");

  ffs_plan_s* p = new ffs_plan_s();
  p->opt = o;
  // auto: deferred for float32 bulk with the adaptive guard alone (at most
  // 8 units), where flagged draws are rare; split-bfloat16 or a fixed margin
  // can flag several percent of draws, more than the record pool holds, so
  // they keep per-step resolution
  p->deferred_auto = o.path == FFS_PATH_BATCHED && o.resolve == FFS_RESOLVE_AUTO &&
                     o.bulk == FFS_BULK_FP32 && o.guard_delta < 0.0 && o.guard_scale <= 8.0;
  p->deferred = p->deferred_auto ||
                (o.path == FFS_PATH_BATCHED && o.resolve == FFS_RESOLVE_DEFERRED);
  p->g_fixed = o.bulk == FFS_BULK_FP64 ? 0.0 : g_fixed;
  p->g_coef = o.bulk == FFS_BULK_FP64 ? 0.0 : g_coef;
  Dims& d = p->d;
  d.L = (int)L;
  d.N = (int)N;
  d.L_pad = (int)round_up(L, SITE_PAD);
  d.Np = (int)round_up(N, 32);
  d.ldu = (int)N;
  d.Kg = cplx ? 2 * d.Np : d.Np;
  d.cplx = cplx ? 1 : 0;
  d.bulk64 = o.bulk == FFS_BULK_FP64 ? 1 : 0;
  d.bf16 = o.bulk == FFS_BULK_SPLIT_BF16 ? 1 : 0;
  (void)hipGetDevice(&p->device);

  const size_t es = cplx ? 16 : 8;
  std::vector<double> u64((size_t)L * N * (cplx ? 2 : 1));
  std::vector<double> u64t((size_t)N * d.L_pad * (cplx ? 2 : 1), 0.0);
  std::vector<float> ub((size_t)d.Kg * d.L_pad, 0.0f);
  for (int64_t i = 0; i < L; ++i)
    for (int64_t j = 0; j < N; ++j) {
      const double re = cplx ? H[(i * ldu + j) * 2] : H[i * ldu + j];
      const double im = cplx ? H[(i * ldu + j) * 2 + 1] : 0.0;
      if (cplx) {
        u64[(i * N + j) * 2] = re;
        u64[(i * N + j) * 2 + 1] = im;
        u64t[((size_t)j * d.L_pad + i) * 2] = re;
        u64t[((size_t)j * d.L_pad + i) * 2 + 1] = im;
        ub[(size_t)j * d.L_pad + i] = (float)re;
        ub[(size_t)(d.Np + j) * d.L_pad + i] = (float)im;
      } else {
        u64[i * N + j] = re;
        u64t[(size_t)j * d.L_pad + i] = re;
        ub[(size_t)j * d.L_pad + i] = (float)re;
      }
    }
  // split-bfloat16 copy: head = bf16(x), tail = bf16(x - head), chunk-major
  std::vector<uint16_t> ubf;
  if (d.bf16) {
    const size_t one = (size_t)d.Kg * d.L_pad;
    ubf.assign(2 * one, 0);
    for (int k = 0; k < d.Kg; ++k)
      for (int i = 0; i < d.L; ++i) {
        const int j = k < d.Np ? k : k - d.Np;
        if (j >= d.N) continue;
        const double v = cplx ? H[(i * ldu + j) * 2 + (k < d.Np ? 0 : 1)] : H[i * ldu + j];
        const uint16_t hb = bf16_bits((float)v);
        const uint16_t lb = bf16_bits((float)(v - (double)bf16_value(hb)));
        const size_t at = ((size_t)(k / 32) * d.L_pad + i) * 32 + (k % 32);
        ubf[at] = hb;
        ubf[one + at] = lb;
      }
  }
  // Metropolis starting site per column: the first row of largest |U[., c]|^2
  std::vector<int32_t> anchor((size_t)N, 0);
  for (int64_t j = 0; j < N; ++j) {
    double best = -1.0;
    for (int64_t i = 0; i < L; ++i) {
      const double re = cplx ? H[(i * ldu + j) * 2] : H[i * ldu + j];
      const double im = cplx ? H[(i * ldu + j) * 2 + 1] : 0.0;
      const double a2 = re * re + im * im;
      if (a2 > best) {
        best = a2;
        anchor[j] = (int32_t)i;
      }
    }
  }
  auto cleanup = [&](ffs_status st) {
    (void)hipFree(p->u64);
    (void)hipFree(p->u64t);
    (void)hipFree(p->ubulk);
    (void)hipFree(p->ubf);
    (void)hipFree(p->anchor);
    delete p;
    return st;
  };
  hipError_t e;
  if ((e = hipMalloc(&p->anchor, (size_t)N * 4)) != hipSuccess ||
      (e = hipMemcpy(p->anchor, anchor.data(), (size_t)N * 4, hipMemcpyHostToDevice)) != hipSuccess)
    return cleanup(fail(FFS_ERR_OUT_OF_MEMORY, "plan allocation: %s", hipGetErrorString(e)));
  if ((e = hipMalloc(&p->u64, (size_t)L * N * es)) != hipSuccess ||
      (e = hipMalloc(&p->u64t, (size_t)N * d.L_pad * es)) != hipSuccess ||
      (e = hipMalloc(&p->ubulk, ub.size() * 4)) != hipSuccess ||
      (d.bf16 && (e = hipMalloc(&p->ubf, ubf.size() * 2)) != hipSuccess))
    return cleanup(fail(FFS_ERR_OUT_OF_MEMORY, "plan allocation: %s", hipGetErrorString(e)));
  if ((e = hipMemcpy(p->u64, u64.data(), (size_t)L * N * es, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(p->u64t, u64t.data(), (size_t)N * d.L_pad * es, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(p->ubulk, ub.data(), ub.size() * 4, hipMemcpyHostToDevice)) != hipSuccess ||
      (d.bf16 && (e = hipMemcpy(p->ubf, ubf.data(), ubf.size() * 2, hipMemcpyHostToDevice)) != hipSuccess))
    return cleanup(fail(FFS_ERR_HIP, "plan upload: %s", hipGetErrorString(e)));
  if ((e = hipEventCreateWithFlags(&p->last_event, hipEventDisableTiming)) != hipSuccess)
    return cleanup(fail(FFS_ERR_HIP, "event: %s", hipGetErrorString(e)));
  *out = p;
  return FFS_OK;
}

static ffs_status replay_listed(ffs_plan_s* p, Slot* sl, uint64_t seed, int n_keep,
                                const int listed[2], int32_t* x_out, double* logdet_out,
                                hipStream_t st);

// deferred: flagged draws are recorded and checked at the end of the call
// (one launch per step and half instead of three; the call then waits for
// the device to learn whether any sample needs a replay).  Needs the slot's
// record buffers.
static ffs_status run_batched(ffs_plan_s* p, Slot* sl, uint64_t seed,
                              uint64_t first, int S, int n_keep,
                              int n_forced, int32_t* x_out, double* logdet_out,
                              hipStream_t st, bool timed = true,
                              const Dims* dims = nullptr, bool deferred = false) {
  const Dims& d = dims ? *dims : p->d;
  // Two halves when the batch is large enough -- and always when it does not
  // fit the first buffer alone (a ragged last chunk after chunks that were
  // split, whose buffers are sized for half a chunk).
  const bool two = sl->w2.S_pad > 0 && ((p->opt.overlap && split_batch(S)) || S > sl->w.S_pad);
  const int SA = two ? first_half(S) : S;
  if (SA > sl->w.S_pad || (two && S - SA > sl->w2.S_pad))
    return fail(FFS_ERR_INVALID_ARG, "internal: batch of %d samples exceeds its working memory", S);
  hipStream_t sb = st;
  if (two) {
    if (!sl->s2) {
      HIP_OK(hipStreamCreateWithFlags(&sl->s2, hipStreamNonBlocking));
      HIP_OK(hipEventCreateWithFlags(&sl->ev_fork, hipEventDisableTiming));
      HIP_OK(hipEventCreateWithFlags(&sl->ev_phase, hipEventDisableTiming));
      HIP_OK(hipEventCreateWithFlags(&sl->ev_join, hipEventDisableTiming));
    }
    sb = sl->s2;
    HIP_OK(hipEventRecord(sl->ev_fork, st));
    HIP_OK(hipStreamWaitEvent(sb, sl->ev_fork, 0));
  }
  struct Half {
    const Work* w;
    int S;
    uint64_t first;
    hipStream_t st;
    int32_t* x;
    double* ld;
  };
  const Half h[2] = {
      {&sl->w, SA, first, st, x_out, logdet_out},
      {&sl->w2, S - SA, first + (uint64_t)SA, sb,
       x_out ? x_out + (size_t)SA * n_keep : nullptr,
       logdet_out ? logdet_out + SA : nullptr}};
  const int nh = two ? 2 : 1;
  const bool defer = deferred && n_forced == 0 && sl->w.rec_cap > 0 &&
                     (!two || sl->w2.rec_cap > 0);
  for (int k = 0; k < nh; ++k) {
    launch_init(d, *h[k].w, h[k].S, h[k].st);
    {
      Timed tm(p, h[k].st, FFS_K_FACTOR, timed);
      launch_factor(d, *h[k].w, p->u64, h[k].S, -1, 0, n_keep, seed, h[k].first, h[k].st);
    }
    if (two && k == 0) {  // start the second half one factor launch later
      HIP_OK(hipEventRecord(sl->ev_phase, st));
      HIP_OK(hipStreamWaitEvent(sb, sl->ev_phase, 0));
    }
  }
  for (int t = 0; t < n_keep; ++t) {
    for (int k = 0; k < nh; ++k) {
      const Work& w = *h[k].w;
      hipStream_t s = h[k].st;
      {
        Timed tm(p, s, FFS_K_WEIGHTS, timed, true);
        unsigned long long* stamp = take_stamp(p, tm.a != nullptr);
        launch_weights(d, w, p->ubulk, p->ubf, h[k].S, s, tm.a, tm.b, stamp);
      }
      const bool closes = t + 1 < n_keep && factor_closes_block(t);
      const int t_solve = (t + 1 < n_keep) ? t + 1 : -1;
      if (defer) {
        Timed tm(p, s, closes ? FFS_K_FACTOR_BLOCK : FFS_K_FACTOR, timed);
        launch_drawfactor(d, w, p->u64, h[k].S, t, t_solve, n_keep, seed, h[k].first,
                          p->g_fixed, p->g_coef, k == 0 ? 0 : SA, s);
        continue;
      }
      {
        Timed tm(p, s, FFS_K_DRAW, timed);
        launch_draw(d, w, h[k].S, t, seed, h[k].first, p->g_fixed, p->g_coef, n_forced, s);
      }
      {
        Timed tm(p, s, FFS_K_REPAIR, timed);
        launch_repair(d, w, p->u64t, h[k].S, t, seed, h[k].first, s);
      }
      {
        Timed tm(p, s, closes ? FFS_K_FACTOR_BLOCK : FFS_K_FACTOR, timed);
        launch_factor(d, w, p->u64, h[k].S, t, t_solve, n_keep, seed, h[k].first, s);
      }
    }
  }
  for (int k = 0; k < nh; ++k) {
    if (defer) {
      Timed tm(p, h[k].st, FFS_K_REPAIR, timed);
      launch_check_records(d, *h[k].w, p->u64t, seed, h[k].first, k == 0 ? 0 : SA, h[k].st);
    }
    if (h[k].x) launch_copy_out(d, *h[k].w, h[k].S, n_keep, h[k].x, h[k].ld, h[k].st);
  }
  if (two) {
    HIP_OK(hipEventRecord(sl->ev_join, sb));
    HIP_OK(hipStreamWaitEvent(st, sl->ev_join, 0));
  }
  HIP_OK(hipGetLastError());
  if (defer) {
    // the samples whose recorded draws moved (or found no record slot)
    if (!sl->listed_host) HIP_OK(hipHostMalloc((void**)&sl->listed_host, 16, hipHostMallocDefault));
    sl->listed_host[0] = sl->listed_host[1] = 0;
    for (int k = 0; k < nh; ++k)
      HIP_OK(hipMemcpyAsync(sl->listed_host + k, h[k].w->rec_ctl + 1, 4, hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    const int listed[2] = {sl->listed_host[0], sl->listed_host[1]};
    if (listed[0] + listed[1] > 0) {
      if (p->deferred_auto) p->deferred = false;
      return replay_listed(p, sl, seed, n_keep, listed, x_out, logdet_out, st);
    }
  }
  return FFS_OK;
}

// Replays, with per-step resolution, the samples a deferred call listed
// (their rows and Philox indices were written by the device into the two
// half-batches' lists) and scatters their rows into the call's output.
static ffs_status replay_listed(ffs_plan_s* p, Slot* sl, uint64_t seed, int n_keep,
                                const int listed[2], int32_t* x_out, double* logdet_out,
                                hipStream_t st) {
  const int n = listed[0] + listed[1];
  if (!sl->replay) sl->replay = new Slot();
  Slot* rs = sl->replay;
  const int need = (int)round_up(n, SAMPLE_PAD);
  if (rs->S_cap < need) {
    free_slot(rs);
    ffs_status e;
    if ((e = alloc_work(p, rs, rs->w, need)) != FFS_OK) return e;
    rs->S_cap = need;
  }
  Work& rw = rs->w;
  if (!sl->replayed) {  // the call's first replay: its counters start at zero
    HIP_OK(hipMemsetAsync(rw.ctl, 0, 256, st));
    HIP_OK(hipMemsetAsync(rw.counters, 0, 256, st));
  }
  const Work* hw[2] = {&sl->w, &sl->w2};
  int at = 0;
  for (int k = 0; k < 2; ++k) {
    if (listed[k] == 0) continue;
    HIP_OK(hipMemcpyAsync(rw.rep_sid + at, hw[k]->rep_sid, (size_t)listed[k] * 8,
                          hipMemcpyDeviceToDevice, st));
    HIP_OK(hipMemcpyAsync(rw.rep_row + at, hw[k]->rep_row, (size_t)listed[k] * 4,
                          hipMemcpyDeviceToDevice, st));
    at += listed[k];
  }
  rw.sid = rw.rep_sid;  // the replay batch's samples are the listed ones
  ffs_status e;
  if ((e = run_batched(p, rs, seed, 0, n, n_keep, 0, nullptr, nullptr, st, false)) != FFS_OK)
    return e;
  if (x_out) launch_scatter_out(p->d, rw, n, n_keep, rw.rep_row, x_out, logdet_out, st);
  HIP_OK(hipGetLastError());
  sl->replayed = true;
  return FFS_OK;
}

static ffs_status sample_impl(ffs_plan_t p, int64_t n_keep, uint64_t seed,
                              uint64_t first, int64_t n, int32_t* x_dev,
                              double* logdet_dev, void* stream) {
  if (!p) return fail(FFS_ERR_INVALID_ARG, "plan is NULL");
  if (n < 0) return fail(FFS_ERR_INVALID_ARG, "n_samples < 0");
  if (n_keep < 0 || n_keep > p->d.N) return fail(FFS_ERR_INVALID_ARG, "n_keep out of range");
  if (n == 0 || n_keep == 0) return FFS_OK;
  if (!x_dev) return fail(FFS_ERR_INVALID_ARG, "x_dev is NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  Slot* sl = get_slot(p, st);
  const Dims& d = p->d;
  int64_t chunk = p->opt.max_batch;
  if (p->opt.path == FFS_PATH_BATCHED && p->opt.hbm_budget) {
    while (chunk > SAMPLE_PAD &&
           slot_bytes(d, (int)round_up(chunk, SAMPLE_PAD), p->deferred.load()) > p->opt.hbm_budget)
      chunk /= 2;
    if (slot_bytes(d, (int)round_up(chunk, SAMPLE_PAD), p->deferred.load()) > p->opt.hbm_budget)
      return fail(FFS_ERR_OUT_OF_MEMORY, "working memory for %lld samples exceeds hbm_budget",
                  (long long)chunk);
  }
  if (p->opt.path == FFS_PATH_PLAIN) chunk = 1;
  const int S0 = (int)(n < chunk ? n : chunk);
  ffs_status s;
  const bool defer = p->deferred;
  if ((s = ensure_slot(p, sl, S0, defer)) != FFS_OK) return s;
  sl->replayed = false;
  if (p->opt.path == FFS_PATH_PLAIN && !sl->plain_scratch) {
    HIP_OK(hipMalloc(&sl->plain_scratch, plain_scratch_bytes(d)));
    sl->allocs.push_back(sl->plain_scratch);
  }
  HIP_OK(hipMemsetAsync(sl->w.ctl, 0, 256, st));
  HIP_OK(hipMemsetAsync(sl->w.counters, 0, 256, st));
  if (sl->w2.S_pad > 0) {
    HIP_OK(hipMemsetAsync(sl->w2.ctl, 0, 256, st));
    HIP_OK(hipMemsetAsync(sl->w2.counters, 0, 256, st));
  }
  for (int64_t off = 0; off < n; off += chunk) {
    const int S = (int)((n - off) < chunk ? (n - off) : chunk);
    int32_t* xo = x_dev + off * n_keep;
    double* lo = logdet_dev ? logdet_dev + off : nullptr;
    if (p->opt.path == FFS_PATH_PLAIN) {
      Timed tm(p, st, FFS_K_PLAIN);
      launch_plain(d, p->u64, p->u64t, p->ubulk, seed, first + off,
                   (int)n_keep, p->g_fixed, p->g_coef, sl->plain_scratch, xo, lo,
                   sl->w.ctl, sl->w.counters, st);
    } else {
      if ((s = run_batched(p, sl, seed, first + off, S, (int)n_keep, 0, xo, lo, st, true,
                           nullptr, defer && p->deferred)) != FFS_OK)
        return s;
    }
  }
  HIP_OK(hipGetLastError());
  HIP_OK(hipEventRecord(p->last_event, st));
  p->last_slot = sl;
  p->last_draws = n * n_keep;
  return FFS_OK;
}

}  // extern "C"

namespace ffsk {

// Working memory of one serving request: one batch of min(n, max_batch)
// samples, reused by its chunks in order.
size_t request_bytes(const ffs_plan_s* p, int64_t n, int* s_chunk) {
  const int64_t chunk = n < p->opt.max_batch ? n : p->opt.max_batch;
  *s_chunk = (int)chunk;
  return carve_work(p->d, nullptr, (int)round_up(chunk, SAMPLE_PAD), nullptr);
}

// Enqueues one request on `st` with working memory at `base` (request_bytes
// bytes, device) and copies its counters and device status to `pinned`
// (host, [0] flagged [1] changed [2] status) at the end.  One stream, no
// timing hooks: the caller may run many of these concurrently.
int run_request(ffs_plan_s* p, void* base, int s_chunk, uint64_t seed,
                uint64_t first, int64_t n, int n_keep, int32_t* x, double* ld,
                hipStream_t st, unsigned long long* pinned) {
  const Dims& d = p->d;
  const int S_pad = (int)round_up(s_chunk, SAMPLE_PAD);
  Slot sl;
  carve_work(d, static_cast<char*>(base), S_pad, &sl.w);
  sl.S_cap = S_pad;
  HIP_OK(hipMemsetAsync(sl.w.gam, 0, (size_t)S_pad * d.Kg * 4, st));
  HIP_OK(hipMemsetAsync(sl.w.ctl, 0, 256, st));
  HIP_OK(hipMemsetAsync(sl.w.counters, 0, 256, st));
  ffs_status s;
  for (int64_t off = 0; off < n; off += s_chunk) {
    const int S = (int)((n - off) < s_chunk ? (n - off) : s_chunk);
    if ((s = run_batched(p, &sl, seed, first + off, S, n_keep, 0, x + off * n_keep,
                         ld ? ld + off : nullptr, st, false)) != FFS_OK)
      return s;
  }
  HIP_OK(hipMemcpyAsync(pinned, sl.w.counters, 16, hipMemcpyDeviceToHost, st));
  HIP_OK(hipMemcpyAsync(pinned + 2, sl.w.ctl, 8, hipMemcpyDeviceToHost, st));
  return FFS_OK;
}

const Dims& plan_dims(const ffs_plan_s* p) { return p->d; }
PlanView plan_view(const ffs_plan_s* p) {
  PlanView v;
  v.d = p->d;
  v.u64 = p->u64;
  v.u64t = p->u64t;
  v.ubulk = p->ubulk;
  v.ubf = p->ubf;
  v.delta = p->g_fixed;
  v.coef = p->g_coef;
  v.max_batch = p->opt.max_batch;
  v.overlap = p->opt.overlap;
  return v;
}
size_t carve(const Dims& d, char* base, int S_pad, Work* w) {
  return carve_work(d, base, S_pad, w);
}
int plan_device(const ffs_plan_s* p) { return p->device; }
int plan_path(const ffs_plan_s* p) { return p->opt.path; }
int set_error(int st, const char* msg) { return fail((ffs_status)st, "%s", msg); }

}  // namespace ffsk

extern "C" {

ffs_status ffs_plan_device(ffs_plan_t* out, const void* U_dev, int64_t L, int64_t N,
                           int64_t ldu, int32_t dtype, const ffs_options* opt) {
  if (!out) return fail(FFS_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!U_dev) return fail(FFS_ERR_INVALID_ARG, "U_dev is NULL");
  if (dtype != FFS_REAL64 && dtype != FFS_COMPLEX128)
    return fail(FFS_ERR_INVALID_ARG, "unknown dtype %d", (int)dtype);
  if (N < 1 || L < N) return fail(FFS_ERR_INVALID_ARG, "need 1 <= N <= L (L=%lld N=%lld)", (long long)L, (long long)N);
  if (ldu < N) return fail(FFS_ERR_INVALID_ARG, "ldu < N");
  if (N > 1024) return fail(FFS_ERR_UNSUPPORTED, "N=%lld above 1024", (long long)N);
  if (L > 65536) return fail(FFS_ERR_UNSUPPORTED, "L=%lld above 65536", (long long)L);
  const size_t n = (size_t)L * ldu * (dtype == FFS_COMPLEX128 ? 2 : 1);
  std::vector<double> host(n);
  HIP_OK(hipMemcpy(host.data(), U_dev, n * sizeof(double), hipMemcpyDeviceToHost));
  return ffs_plan(out, host.data(), L, N, ldu, dtype, opt);
}

ffs_status ffs_sample(ffs_plan_t p, uint64_t seed, uint64_t first_sample,
                      int64_t n_samples, int32_t* x_dev, double* logdet_dev,
                      void* hip_stream) {
  if (!p) return fail(FFS_ERR_INVALID_ARG, "plan is NULL");
  return sample_impl(p, p->d.N, seed, first_sample, n_samples, x_dev,
                     logdet_dev, hip_stream);
}

ffs_status ffs_marginal(ffs_plan_t p, int64_t n_keep, uint64_t seed,
                        uint64_t first_sample, int64_t n_samples,
                        int32_t* x_dev, void* hip_stream) {
  return sample_impl(p, n_keep, seed, first_sample, n_samples, x_dev, nullptr,
                     hip_stream);
}

}  // extern "C"

// ---- allocation-free sampling ----------------------------------------------
// Working memory of ffs_sample_noalloc: a file-scope device array (one copy
// per GPU, held until the process ends).  Host code never passes `scratch`
// itself to a kernel -- in host code that name is a host-side stand-in --
// but the device address hipGetSymbolAddress returns for the current device,
// taken once per device and kept in g_noalloc.
static __device__ __align__(256) char scratch[FFS_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;

struct NoAllocDevice {
  std::once_flag once;
  hipError_t err = hipSuccess;
  char* ptr = nullptr;  // device address of this GPU's copy of `scratch`
  Slot slot;            // views into ptr of the last call (read by ffs_check)
};
NoAllocDevice g_noalloc[kMaxDevices];

__global__ void zero_words_kernel(uint32_t* p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

// Clears n 32-bit words with a kernel (no memset node if the caller
// captures the stream into a graph).
void zero_words(void* p, size_t n, hipStream_t st) {
  const size_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(zero_words_kernel, dim3(blocks < 1024 ? (unsigned)blocks : 1024u),
                     dim3(256), 0, st, static_cast<uint32_t*>(p), n);
}

}  // namespace

extern "C" {

ffs_status ffs_sample_noalloc(ffs_plan_t p, uint64_t seed, uint64_t first_sample,
                              int64_t n, int32_t* x_dev, double* logdet_dev,
                              void* stream) {
  if (!p) return fail(FFS_ERR_INVALID_ARG, "plan is NULL");
  if (n < 0) return fail(FFS_ERR_INVALID_ARG, "n_samples < 0");
  if (p->opt.path != FFS_PATH_BATCHED)
    return fail(FFS_ERR_UNSUPPORTED, "the allocation-free call needs a batched-path plan");
  if (n == 0) return FFS_OK;
  if (!x_dev) return fail(FFS_ERR_INVALID_ARG, "x_dev is NULL");
  int dev = -1;
  HIP_OK(hipGetDevice(&dev));
  if (dev != p->device)
    return fail(FFS_ERR_INVALID_ARG, "plan lives on device %d, current device is %d",
                p->device, dev);
  if (dev < 0 || dev >= kMaxDevices) return fail(FFS_ERR_UNSUPPORTED, "device %d", dev);
  NoAllocDevice& nd = g_noalloc[dev];
  std::call_once(nd.once, [&nd]() {
    void* ptr = nullptr;
    nd.err = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (nd.err == hipSuccess) nd.ptr = static_cast<char*>(ptr);
  });
  if (nd.err != hipSuccess || !nd.ptr)
    return fail(FFS_ERR_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(nd.err));
  const Dims& d = p->d;
  // largest batch whose working memory fits the scratch array
  const int64_t want = round_up(n < p->opt.max_batch ? n : p->opt.max_batch, SAMPLE_PAD);
  int S_pad = 0;
  for (int64_t c = want; c >= SAMPLE_PAD; c -= SAMPLE_PAD)
    if (carve_work(d, nullptr, (int)c, nullptr) <= (size_t)FFS_NOALLOC_SCRATCH_BYTES) {
      S_pad = (int)c;
      break;
    }
  if (S_pad == 0)
    return fail(FFS_ERR_UNSUPPORTED,
                "working memory of one %d-sample batch (%zu bytes) exceeds the %zu-byte "
                "scratch of the allocation-free call", SAMPLE_PAD,
                carve_work(d, nullptr, SAMPLE_PAD, nullptr),
                (size_t)FFS_NOALLOC_SCRATCH_BYTES);
  hipStream_t st = static_cast<hipStream_t>(stream);
  Slot& sl = nd.slot;
  sl.w2 = Work();
  carve_work(d, nd.ptr, S_pad, &sl.w);
  sl.S_cap = S_pad;
  // what must start at zero: Gamma (its padded columns and samples are never
  // written), the flag count / status word and the guard counters
  zero_words(sl.w.gam, (size_t)S_pad * d.Kg, st);
  zero_words(sl.w.ctl, 256 / 4, st);
  zero_words(sl.w.counters, 256 / 4, st);
  ffs_status s;
  for (int64_t off = 0; off < n; off += S_pad) {
    const int S = (int)((n - off) < S_pad ? (n - off) : S_pad);
    if ((s = run_batched(p, &sl, seed, first_sample + off, S, d.N, 0, x_dev + off * d.N,
                         logdet_dev ? logdet_dev + off : nullptr, st, false)) != FFS_OK)
      return s;
  }
  HIP_OK(hipGetLastError());
  HIP_OK(hipEventRecord(p->last_event, st));
  p->last_slot = &sl;
  p->last_draws = n * d.N;
  return FFS_OK;
}

// Column-subset run; sid (device, nullable) gives each sample's Philox
// sample index (first_sample + s when null).
static ffs_status subsets_run(ffs_plan_t p, int64_t k, const int32_t* cols_dev,
                              uint64_t seed, uint64_t first_sample, int64_t n,
                              int32_t* x_dev, double* logdet_dev, hipStream_t st,
                              const uint64_t* sid) {
  Dims dk = p->d;  // k particles; U keeps its N columns (row stride, contraction K)
  dk.N = (int)k;
  const int64_t chunk = n < p->opt.max_batch ? n : p->opt.max_batch;
  const int S_pad = (int)round_up(chunk, SAMPLE_PAD);
  Slot* sl;
  {
    std::lock_guard<std::mutex> g(p->mu);
    auto it = p->subset_slots.find(st);
    sl = it == p->subset_slots.end() ? (p->subset_slots[st] = new Slot()) : it->second;
    int& kcap = p->subset_kcap[st];
    if (S_pad > sl->S_cap || k > kcap) {
      free_slot(sl);
      kcap = kcap > (int)k ? kcap : (int)k;
      const int scap = S_pad > sl->S_cap ? S_pad : sl->S_cap;
      Dims dc = dk;
      dc.N = kcap;
      void* base = nullptr;
      const size_t bytes = carve_work(dc, nullptr, scap, nullptr);
      HIP_OK(hipMalloc(&base, bytes));
      sl->allocs.push_back(base);
      sl->S_cap = scap;
    }
  }
  carve_work(dk, static_cast<char*>(sl->allocs[0]), S_pad, &sl->w);
  sl->w.cmap = sl->w.cmap_buf;
  HIP_OK(hipMemsetAsync(sl->w.ctl, 0, 256, st));
  HIP_OK(hipMemsetAsync(sl->w.counters, 0, 256, st));
  ffs_status s;
  for (int64_t off = 0; off < n; off += chunk) {
    const int S = (int)((n - off) < chunk ? (n - off) : chunk);
    sl->w.sid = sid ? sid + off : nullptr;
    // Gamma rows are dense over U's columns: clear what other subsets left
    HIP_OK(hipMemsetAsync(sl->w.gam, 0, (size_t)S_pad * dk.Kg * 4, st));
    launch_colmap(dk, sl->w, cols_dev + off * k, S, st);
    s = run_batched(p, sl, seed, first_sample + off, S, (int)k, 0, x_dev + off * k,
                    logdet_dev ? logdet_dev + off : nullptr, st, true, &dk);
    sl->w.sid = nullptr;
    if (s != FFS_OK) return s;
  }
  HIP_OK(hipGetLastError());
  HIP_OK(hipEventRecord(p->last_event, st));
  p->last_slot = sl;
  return FFS_OK;
}

ffs_status ffs_sample_subsets(ffs_plan_t p, int64_t k, const int32_t* cols_dev,
                              uint64_t seed, uint64_t first_sample,
                              int64_t n, int32_t* x_dev, double* logdet_dev,
                              void* stream) {
  if (!p) return fail(FFS_ERR_INVALID_ARG, "plan is NULL");
  if (p->opt.path != FFS_PATH_BATCHED)
    return fail(FFS_ERR_INVALID_ARG, "column subsets need a batched-path plan");
  if (k < 1 || k > p->d.N) return fail(FFS_ERR_INVALID_ARG, "k out of range");
  if (n < 0) return fail(FFS_ERR_INVALID_ARG, "n_samples < 0");
  if (n == 0) return FFS_OK;
  if (!cols_dev || !x_dev) return fail(FFS_ERR_INVALID_ARG, "NULL argument");
  hipStream_t st = static_cast<hipStream_t>(stream);
  ffs_status s = subsets_run(p, k, cols_dev, seed, first_sample, n, x_dev, logdet_dev, st, nullptr);
  if (s == FFS_OK) p->last_draws = n * k;
  return s;
}

ffs_status ffs_sample_dpp(ffs_plan_t p, const int32_t* cols_dev, const int32_t* sizes_dev,
                          uint64_t seed, uint64_t first_sample, int64_t n, int32_t* x_dev,
                          double* logdet_dev, void* stream) {
  if (!p) return fail(FFS_ERR_INVALID_ARG, "plan is NULL");
  if (p->opt.path != FFS_PATH_BATCHED)
    return fail(FFS_ERR_INVALID_ARG, "DPP runs need a batched-path plan");
  if (n < 0) return fail(FFS_ERR_INVALID_ARG, "n_samples < 0");
  if (n == 0) return FFS_OK;
  if (!cols_dev || !sizes_dev || !x_dev) return fail(FFS_ERR_INVALID_ARG, "NULL argument");
  if (n > ((int64_t)1 << 31) - 1) return fail(FFS_ERR_UNSUPPORTED, "n_samples above 2^31 - 1");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int N = p->d.N;
  std::vector<int32_t> sz((size_t)n);
  HIP_OK(hipMemcpyAsync(sz.data(), sizes_dev, n * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  // samples grouped by size (counting sort, ascending sample order inside a group)
  std::vector<int64_t> start((size_t)N + 2, 0);
  for (int64_t i = 0; i < n; ++i) {
    if (sz[i] < 0 || sz[i] > N)
      return fail(FFS_ERR_INVALID_ARG, "size %d of sample %lld outside [0, %d]", (int)sz[i],
                  (long long)i, N);
    ++start[sz[i] + 1];
  }
  for (int k = 0; k <= N; ++k) start[k + 1] += start[k];
  std::vector<int32_t> pos((size_t)n);
  std::vector<uint64_t> ids((size_t)n);
  {
    std::vector<int64_t> fill(start.begin(), start.end() - 1);
    for (int64_t i = 0; i < n; ++i) {
      const int64_t j = fill[sz[i]]++;
      pos[j] = (int32_t)i;
      ids[j] = first_sample + (uint64_t)i;
    }
  }
  int kmax = 0;
  for (int k = N; k >= 1; --k)
    if (start[k + 1] > start[k]) {
      kmax = k;
      break;
    }
  // device scratch: positions, Philox indices, gathered columns, bucket draws
  const size_t b_pos = round_up(n * 4, 256), b_ids = round_up(n * 8, 256);
  const size_t b_cols = round_up(n * (int64_t)(kmax > 0 ? kmax : 1) * 4, 256);
  const size_t b_ld = round_up(n * 8, 256);
  char* buf = nullptr;
  HIP_OK(hipMallocAsync((void**)&buf, b_pos + b_ids + 2 * b_cols + b_ld + 256, st));
  int32_t* dpos = reinterpret_cast<int32_t*>(buf);
  uint64_t* dids = reinterpret_cast<uint64_t*>(buf + b_pos);
  int32_t* dcols = reinterpret_cast<int32_t*>(buf + b_pos + b_ids);
  int32_t* dx = reinterpret_cast<int32_t*>(buf + b_pos + b_ids + b_cols);
  double* dld = reinterpret_cast<double*>(buf + b_pos + b_ids + 2 * b_cols);
  // status word and (flagged, changed) counters summed over the size groups
  unsigned long long* acc = reinterpret_cast<unsigned long long*>(buf + b_pos + b_ids +
                                                                  2 * b_cols + b_ld);
  HIP_OK(hipMemsetAsync(acc, 0, 256, st));
  HIP_OK(hipMemcpyAsync(dpos, pos.data(), n * 4, hipMemcpyHostToDevice, st));
  HIP_OK(hipMemcpyAsync(dids, ids.data(), n * 8, hipMemcpyHostToDevice, st));
  launch_fill_rows(x_dev, logdet_dev, (int)n, N, st);
  // Size groups are independent (each sample keeps its own Philox stream),
  // so they run round-robin on the caller's stream and the plan's DPP
  // streams, each in its own rows of the staging buffers.
  std::lock_guard<std::mutex> dpp_lock(p->dpp_mu);
  constexpr int NS = ffs_plan_s::kDppStreams;
  if (!p->dpp_fork) {
    HIP_OK(hipEventCreateWithFlags(&p->dpp_fork, hipEventDisableTiming));
    for (int i = 0; i < NS; ++i) {
      HIP_OK(hipStreamCreateWithFlags(&p->dpp_st[i], hipStreamNonBlocking));
      HIP_OK(hipEventCreateWithFlags(&p->dpp_join[i], hipEventDisableTiming));
    }
  }
  HIP_OK(hipEventRecord(p->dpp_fork, st));
  for (int i = 0; i < NS; ++i) HIP_OK(hipStreamWaitEvent(p->dpp_st[i], p->dpp_fork, 0));
  ffs_status s = FFS_OK;
  int64_t draws = 0;
  int g = 0;
  for (int k = 1; k <= N; ++k) {
    const int64_t b0 = start[k], nb = start[k + 1] - start[k];
    if (nb == 0) continue;
    hipStream_t gs = (g % (NS + 1) == 0) ? st : p->dpp_st[g % (NS + 1) - 1];
    ++g;
    int32_t* gc = dcols + b0 * kmax;
    int32_t* gx = dx + b0 * kmax;
    double* gl = logdet_dev ? dld + b0 : nullptr;
    launch_gather_rows(cols_dev, N, dpos + b0, (int)nb, k, gc, gs);
    s = subsets_run(p, k, gc, seed, 0, nb, gx, gl, gs, dids + b0);
    if (s != FFS_OK) break;
    launch_stats_add(p->last_slot->w.ctl, p->last_slot->w.counters, acc, gs);
    launch_scatter_rows(gx, gl, dpos + b0, (int)nb, k, x_dev, N, logdet_dev, gs);
    draws += nb * k;
  }
  for (int i = 0; i < NS; ++i) {
    HIP_OK(hipEventRecord(p->dpp_join[i], p->dpp_st[i]));
    HIP_OK(hipStreamWaitEvent(st, p->dpp_join[i], 0));
  }
  if (s == FFS_OK && p->last_slot && draws > 0) {
    launch_stats_store(acc, p->last_slot->w.ctl, p->last_slot->w.counters, st);
    HIP_OK(hipEventRecord(p->last_event, st));
  }
  HIP_OK(hipFreeAsync(buf, st));
  HIP_OK(hipGetLastError());
  if (s == FFS_OK) p->last_draws = draws;
  return s;
}

ffs_status ffs_sample_mh(ffs_plan_t p, int32_t m_cond, int32_t radius, uint64_t seed,
                         uint64_t first_sample, int64_t n, int32_t* x_dev, double* logdet_dev,
                         int64_t* accepted_out, void* stream) {
  if (!p) return fail(FFS_ERR_INVALID_ARG, "plan is NULL");
  if (p->opt.path != FFS_PATH_BATCHED)
    return fail(FFS_ERR_INVALID_ARG, "Metropolis runs need a batched-path plan");
  if (m_cond < 0 || radius < 0) return fail(FFS_ERR_INVALID_ARG, "m_cond and radius must be >= 0");
  if (radius > p->d.L / 2) return fail(FFS_ERR_INVALID_ARG, "radius above L/2");
  if (n < 0) return fail(FFS_ERR_INVALID_ARG, "n_samples < 0");
  if (accepted_out) *accepted_out = 0;
  if (n == 0) return FFS_OK;
  if (!x_dev) return fail(FFS_ERR_INVALID_ARG, "x_dev is NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  Slot* sl = get_slot(p, st);
  const Dims& d = p->d;
  const int64_t chunk = n < p->opt.max_batch ? n : p->opt.max_batch;
  ffs_status s;
  if ((s = ensure_slot(p, sl, (int)chunk)) != FFS_OK) return s;
  const Work& w = sl->w;  // one buffer; a chunk larger than it runs in pieces
  HIP_OK(hipMemsetAsync(w.ctl, 0, 256, st));
  HIP_OK(hipMemsetAsync(w.counters, 0, 256, st));
  if (sl->w2.S_pad > 0) {  // unused here, but read by ffs_check
    HIP_OK(hipMemsetAsync(sl->w2.ctl, 0, 256, st));
    HIP_OK(hipMemsetAsync(sl->w2.counters, 0, 256, st));
  }
  const int N = d.N;
  for (int64_t off = 0; off < n; off += w.S_pad) {
    const int S = (int)((n - off) < w.S_pad ? (n - off) : w.S_pad);
    const uint64_t first = first_sample + off;
    launch_init(d, w, S, st);
    {
      Timed tm(p, st, FFS_K_FACTOR);
      launch_factor(d, w, p->u64, S, -1, 0, N, seed, first, st);
    }
    for (int t = 0; t < N; ++t) {
      {
        Timed tm(p, st, FFS_K_DRAW);
        launch_mh(d, w, p->u64, p->anchor, S, t, m_cond, radius, seed, first, st);
      }
      const bool closes = t + 1 < N && factor_closes_block(t);
      Timed tm(p, st, closes ? FFS_K_FACTOR_BLOCK : FFS_K_FACTOR);
      launch_factor(d, w, p->u64, S, t, (t + 1 < N) ? t + 1 : -1, N, seed, first, st);
    }
    launch_copy_out(d, w, S, N, x_dev + off * N, logdet_dev ? logdet_dev + off : nullptr, st);
  }
  HIP_OK(hipGetLastError());
  HIP_OK(hipEventRecord(p->last_event, st));
  p->last_slot = sl;
  p->last_draws = n * N;
  if (accepted_out) {
    unsigned long long c[3] = {0, 0, 0};
    HIP_OK(hipMemcpyAsync(c, w.counters, sizeof c, hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    *accepted_out = (int64_t)c[2];
  }
  return FFS_OK;
}

ffs_status ffs_check(ffs_plan_t p, ffs_stats_t* stats) {
  if (!p) return fail(FFS_ERR_INVALID_ARG, "plan is NULL");
  if (stats) memset(stats, 0, sizeof *stats);
  if (!p->last_slot) return FFS_OK;
  HIP_OK(hipEventSynchronize(p->last_event));
  int32_t ctl[2] = {0, 0};
  unsigned long long cnt[2] = {0, 0};
  const Slot* ls = p->last_slot;
  const Work* ws[3] = {&ls->w, &ls->w2, ls->replayed && ls->replay ? &ls->replay->w : nullptr};
  for (const Work* w : ws) {
    if (!w || w->S_pad == 0) continue;
    int32_t c2[2];
    unsigned long long n2[2];
    HIP_OK(hipMemcpy(c2, w->ctl, sizeof c2, hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(n2, w->counters, sizeof n2, hipMemcpyDeviceToHost));
    ctl[1] |= c2[1];
    cnt[0] += n2[0];
    cnt[1] += n2[1];
  }
  if (stats) {
    stats->draws = p->last_draws;
    stats->flagged = (int64_t)cnt[0];
    stats->changed = (int64_t)cnt[1];
    stats->device_status = (ctl[1] & DEV_BADCOLS)     ? FFS_ERR_INVALID_ARG
                           : (ctl[1] & DEV_NUMERICAL) ? FFS_ERR_NUMERICAL
                                                      : FFS_OK;
  }
  if (ctl[1] & DEV_BADCOLS)
    return fail(FFS_ERR_INVALID_ARG, "a column subset had a column out of range or repeated");
  if (ctl[1] & DEV_NUMERICAL)
    return fail(FFS_ERR_NUMERICAL, "device reported a zero/non-finite total weight or pivot");
  return FFS_OK;
}

ffs_status ffs_conditional(ffs_plan_t p, uint64_t seed, uint64_t sample,
                           int64_t k, const int32_t* prefix_host,
                           double* w_host) {
  if (!p || !w_host) return fail(FFS_ERR_INVALID_ARG, "NULL argument");
  const Dims& d = p->d;
  if (k < 1 || k > d.N) return fail(FFS_ERR_INVALID_ARG, "k out of range");
  if (k > 1 && !prefix_host) return fail(FFS_ERR_INVALID_ARG, "prefix is NULL");
  for (int64_t i = 0; i + 1 < k; ++i) {
    if (prefix_host[i] < 0 || prefix_host[i] >= d.L)
      return fail(FFS_ERR_INVALID_ARG, "prefix site out of range");
    for (int64_t j = 0; j < i; ++j)
      if (prefix_host[j] == prefix_host[i])
        return fail(FFS_ERR_INVALID_ARG, "prefix repeats a site");
  }
  hipStream_t st = nullptr;
  Slot local;
  ffs_status s;
  if ((s = ensure_slot(p, &local, 1)) != FFS_OK) return s;
  const Work& w = local.w;
  auto done = [&](ffs_status r) {
    (void)hipDeviceSynchronize();
    free_slot(&local);
    return r;
  };
  if (k > 1 &&
      hipMemcpy(w.forced, prefix_host, (size_t)(k - 1) * 4, hipMemcpyHostToDevice) != hipSuccess)
    return done(fail(FFS_ERR_HIP, "prefix upload failed"));
  launch_init(d, w, 1, st);
  launch_factor(d, w, p->u64, 1, -1, 0, (int)k, seed, sample, st);
  for (int t = 0; t < k; ++t) {
    launch_weights(d, w, p->ubulk, p->ubf, 1, st);
    if (t == k - 1) break;
    launch_draw(d, w, 1, t, seed, sample, 0.0, 0.0, (int)k - 1, st);
    launch_factor(d, w, p->u64, 1, t, t + 1, (int)k, seed, sample, st);
  }
  std::vector<float> wh(d.L_pad);
  std::vector<double> bs((size_t)d.L_pad / 32 * w.S_pad);
  if (hipMemcpy(wh.data(), w.wh, wh.size() * 4, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(bs.data(), w.bsum, bs.size() * 8, hipMemcpyDeviceToHost) != hipSuccess)
    return done(fail(FFS_ERR_HIP, "readback failed"));
  double T = 0.0;
  for (int b = 0; b < d.L_pad / 32; ++b) T += bs[b];
  if (!(T > 0.0)) return done(fail(FFS_ERR_NUMERICAL, "zero total weight"));
  for (int x = 0; x < d.L; ++x) w_host[x] = (double)wh[x] / T;
  return done(FFS_OK);
}

ffs_status ffs_density(ffs_plan_t p, double* rho_host) {
  if (!p || !rho_host) return fail(FFS_ERR_INVALID_ARG, "NULL argument");
  double* rho = nullptr;
  HIP_OK(hipMalloc(&rho, (size_t)p->d.L * 8));
  launch_density(p->d, p->ubulk, rho, nullptr);
  hipError_t e = hipMemcpy(rho_host, rho, (size_t)p->d.L * 8, hipMemcpyDeviceToHost);
  (void)hipFree(rho);
  if (e != hipSuccess) return fail(FFS_ERR_HIP, "density readback: %s", hipGetErrorString(e));
  return FFS_OK;
}

ffs_status ffs_set_timing(ffs_plan_t p, int32_t enable) {
  if (!p) return fail(FFS_ERR_INVALID_ARG, "plan is NULL");
  p->timing = enable != 0 ? (1u << FFS_K_COUNT) - 1u : 0u;
  return ensure_stamps(p);
}

ffs_status ffs_set_timing_classes(ffs_plan_t p, uint32_t class_mask) {
  if (!p) return fail(FFS_ERR_INVALID_ARG, "plan is NULL");
  if (class_mask >> FFS_K_COUNT)
    return fail(FFS_ERR_INVALID_ARG, "class mask 0x%x names no kernel class", class_mask);
  p->timing = class_mask;
  return ensure_stamps(p);
}

ffs_status ffs_set_timing_stride(ffs_plan_t p, int32_t stride) {
  if (!p) return fail(FFS_ERR_INVALID_ARG, "plan is NULL");
  if (stride < 1) return fail(FFS_ERR_INVALID_ARG, "timing stride %d < 1", stride);
  p->timing_stride = stride;
  for (int c = 0; c < FFS_K_COUNT; ++c) p->timing_seen[c] = 0;
  return FFS_OK;
}

ffs_status ffs_kernel_times(ffs_plan_t p, double* ms, int64_t* launches) {
  if (!p || !ms) return fail(FFS_ERR_INVALID_ARG, "NULL argument");
  for (int c = 0; c < FFS_K_COUNT; ++c) {
    ms[c] = 0.0;
    if (launches) launches[c] = 0;
  }
  for (auto& r : p->recs) {
    HIP_OK(hipEventSynchronize(r.b));
    float t = 0.f;
    HIP_OK(hipEventElapsedTime(&t, r.a, r.b));
    ms[r.cls] += t;
    if (launches) launches[r.cls] += 1;
    p->pool.push_back(r.a);
    p->pool.push_back(r.b);
  }
  p->recs.clear();
  return FFS_OK;
}

ffs_status ffs_kernel_spans(ffs_plan_t p, double* ms, int64_t* launches) {
  if (!p || !ms) return fail(FFS_ERR_INVALID_ARG, "NULL argument");
  *ms = 0.0;
  if (launches) *launches = 0;
  if (p->kstamp_n == 0) return FFS_OK;
  HIP_OK(hipDeviceSynchronize());
  std::vector<unsigned long long> st(2 * (size_t)p->kstamp_n);
  HIP_OK(hipMemcpy(st.data(), p->kstamp, st.size() * 8, hipMemcpyDeviceToHost));
  for (int i = 0; i < p->kstamp_n; ++i) {
    const unsigned long long t0 = st[2 * (size_t)i], t1 = st[2 * (size_t)i + 1];
    if (t1 > t0 && t0 != ~0ull) *ms += (double)(t1 - t0) / p->wall_khz;
  }
  if (launches) *launches = p->kstamp_n;
  HIP_OK(reset_stamps(p, p->kstamp_n));
  p->kstamp_n = 0;
  return FFS_OK;
}

ffs_status ffs_destroy(ffs_plan_t p) {
  if (!p) return FFS_OK;
  (void)hipDeviceSynchronize();
  for (auto& r : p->recs) {
    if (r.a) (void)hipEventDestroy(r.a);
    if (r.b) (void)hipEventDestroy(r.b);
  }
  (void)hipFree(p->kstamp);
  for (auto e : p->pool) (void)hipEventDestroy(e);
  for (auto& kv : p->slots) {
    Slot* sl = kv.second;
    free_slot(sl);
    if (sl->replay) {
      free_slot(sl->replay);
      delete sl->replay;
    }
    if (sl->listed_host) (void)hipHostFree(sl->listed_host);
    if (sl->s2) (void)hipStreamDestroy(sl->s2);
    if (sl->ev_fork) (void)hipEventDestroy(sl->ev_fork);
    if (sl->ev_phase) (void)hipEventDestroy(sl->ev_phase);
    if (sl->ev_join) (void)hipEventDestroy(sl->ev_join);
    delete sl;
  }
  for (auto& kv : p->subset_slots) {
    free_slot(kv.second);
    delete kv.second;
  }
  (void)hipFree(p->u64);
  (void)hipFree(p->u64t);
  (void)hipFree(p->ubulk);
  (void)hipFree(p->ubf);
  (void)hipFree(p->anchor);
  for (int i = 0; i < ffs_plan_s::kDppStreams; ++i) {
    if (p->dpp_st[i]) (void)hipStreamDestroy(p->dpp_st[i]);
    if (p->dpp_join[i]) (void)hipEventDestroy(p->dpp_join[i]);
  }
  if (p->dpp_fork) (void)hipEventDestroy(p->dpp_fork);
  if (p->last_event) (void)hipEventDestroy(p->last_event);
  delete p;
  return FFS_OK;
}

}  // extern "C"
