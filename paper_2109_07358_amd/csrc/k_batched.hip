// Batched-path kernels other than the contraction and the draw: per-call
// init, the per-step factor kernel (one wavefront per sample), copy-out and
// the density hook.
#include "factor_blk.h"
#include "args.h"
#include "draw.h"
#include "ffs_internal.h"

namespace ffsk {

namespace {

// ---------------------------------------------------------------- init ----
__global__ void init_kernel(int32_t* perm, double* logdet, uint32_t* occ,
                            int32_t* ctl, int32_t* rec_ctl, int32_t* div, int S, int N,
                            int nblk) {
  const int s = blockIdx.x;
  if (s >= S) return;
  for (int i = threadIdx.x; i < N; i += blockDim.x) perm[(size_t)s * N + i] = i;
  for (int i = threadIdx.x; i < nblk; i += blockDim.x) occ[(size_t)s * nblk + i] = 0u;
  if (threadIdx.x == 0) {
    logdet[s] = 0.0;
    div[s] = 0;
    if (s == 0) {
      ctl[0] = 0;
      rec_ctl[0] = 0;
      rec_ctl[1] = 0;
    }
  }
}

// -------------------------------------------------------------- factor ----

// Float64 redraw of sample s's flagged draw at step t (redraw slot f): the
// site from the slot's float64 weights and chunk sums (redraw_site); a slot
// with no float64 mass keeps the first draw and reports NUMERICAL.
__device__ inline void redraw_flagged(const FArgs& a, int s, int f, int lane, char* lds) {
  const int nch = a.L_pad / RCHUNK;
  const int t = a.t_upd;
  int site = redraw_site(a.cs + (size_t)f * nch, a.wr + (size_t)f * a.L_pad, a.L_pad, a.seed,
                         sample_index(a.sid, a.first, s), t, lane, lds);
  if (lane == 0) {
    const int nblk = a.L_pad / 32;
    int32_t* xrow = a.xs + (size_t)s * a.N;
    if (site < 0) {
      atomicOr(&a.ctl[1], (int)DEV_NUMERICAL);
      site = xrow[t];
    }
    if (xrow[t] != site) atomicAdd(&a.counters[1], 1ull);
    xrow[t] = site;
    a.occ[(size_t)s * nblk + (site >> 5)] |= 1u << (site & 31);
  }
  lane_fence();  // the redrawn site is read by every lane of the update
}

template <bool C, bool BND>
__device__ inline void factor_sample(const FArgs& a, int s, int lane, char* lds) {
  using X = Cx<C>;
  using T = typename X::T;
  if (s == 0 && lane == 0) a.ctl[0] = 0;  // flag count of the coming draw
  if (a.t_upd >= 0 && a.fslot) {
    const int f = a.fslot[s];
    if (f >= 0) redraw_flagged(a, s, f, lane, lds);
  }
  const int N = a.N;
  BlkSample<C> f;
  T* base = reinterpret_cast<T*>(a.F) + (size_t)s * blk_state_elems(N);
  f.U = reinterpret_cast<const T*>(a.u64);
  f.F = base;
  f.E = f.F + (size_t)N * N;
  f.Z = f.E + (size_t)BB * N;
  f.G = f.Z + (size_t)N * BB;
  f.Gn = f.G + (size_t)N * BB;
  f.Kn = f.Gn + (size_t)N * BB;
  f.Sg = f.Kn + (size_t)N * BB;
  f.SLi = f.Sg + BB * BB;
  f.SP = f.SLi + BB * BB;
  f.Xr = f.SP + BB * BB;
  f.beta = reinterpret_cast<T*>(a.beta) + (size_t)s * N;
  f.perm = a.perm + (size_t)s * N;
  f.xs = a.xs + (size_t)s * N;
  f.logdet = a.logdet + s;
  f.status = a.ctl + 1;
  f.N = N;
  f.ldu = a.ldu;
  f.cmap = a.cmap ? a.cmap + (size_t)s * N : nullptr;
  f.n_steps = a.n_steps;
  f.seed = a.seed;
  f.sample = sample_index(a.sid, a.first, s);
  T* gl;
  blk_wave<C, BND>(f, a.t_upd, a.t_solve, lane, lds, &gl);
  if (a.t_solve < 0) return;
  if (a.gsplit) {  // split-BF16: the contraction's operands, head and tail
    uint16_t* gs = a.gsplit + (size_t)s * 2 * a.Kg;
    auto put = [&](int c, float x) {
      const uint32_t h = bf16_rn(x);
      const int o = (c >> 4) * 32 + (c & 15);
      gs[o] = (uint16_t)h;
      gs[o + 16] = (uint16_t)bf16_rn(x - __uint_as_float(h << 16));
    };
    for (int i = lane; i < N; i += 64) {
      const T v = gl[i];
      const int c = f.cmap ? f.cmap[i] : i;
      put(c, (float)X::re(v));
      if (C) put(a.Np + c, (float)X::im(v));
    }
    return;
  }
  float* g = a.gam + (size_t)s * a.Kg;
  for (int i = lane; i < N; i += 64) {
    const T v = gl[i];
    const int c = f.cmap ? f.cmap[i] : i;
    g[c] = (float)X::re(v);
    if (C) g[a.Np + c] = (float)X::im(v);
  }
}

template <bool C, bool BND>
__global__ __launch_bounds__(64) void factor_kernel(FArgs a) {
  extern __shared__ __align__(16) char lds[];
  factor_sample<C, BND>(a, blockIdx.x, threadIdx.x, lds);
}

// Deferred resolution: the draw of step a.t_upd and the factor update that
// absorbs it in one launch (one wavefront per sample; a flagged draw is
// recorded, not redone, so nothing between the two depends on other
// samples).  The draw's 64 lane totals use the start of the factor's LDS.
template <bool C, bool BND>
__global__ __launch_bounds__(64) void drawfactor_kernel(FArgs a, DArgs d) {
  extern __shared__ __align__(16) char lds[];
  const int s = blockIdx.x, lane = threadIdx.x;
  draw_one<true>(d, s, lane, reinterpret_cast<double*>(lds));
  lane_fence();  // the drawn site and occupancy bit are read by every lane below
  factor_sample<C, BND>(a, s, lane, lds);
}

// Replay rows into the caller's output: row rows[r] of x_out (n_keep wide)
// and logdet_out from row r of the replay batch.
__global__ void scatter_out_kernel(const int32_t* xs, const double* logdet, const int32_t* rows,
                                   int n, int N, int n_keep, int32_t* x_out, double* logdet_out) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)n * n_keep) return;
  const size_t r = i / n_keep, j = i % n_keep;
  x_out[(size_t)rows[r] * n_keep + j] = xs[r * N + j];
  if (logdet_out && j == 0) logdet_out[rows[r]] = logdet[r];
}

// Grouped factor step: one wavefront per (instance, sample) item; the step
// comes from the instance's device-side step counter.  Two launches per
// tick: BND = false takes the instances whose step is a regular one, BND =
// true those closing a 16-step block, so the regular launches keep the small
// register and LDS footprint of the regular instantiation.
template <bool C, bool BND>
__global__ __launch_bounds__(64) void factor_group_kernel(const GInst* inst, GList l) {
  extern __shared__ __align__(16) char lds[];
  const int item = blockIdx.x;  // one (instance, sample) item per workgroup
  if (item >= l.total) return;
  const int k = glist_find(l, item);
  const GInst* I = inst + l.ids[k];
  const int t = I->t;
  if (t < 0 || t >= I->n_keep) return;
  const int t_solve = (t + 1 < I->n_keep) ? t + 1 : -1;
  const bool closes = t_solve >= 0 && (t % BB) == BB - 1;
  if (closes != BND) return;
  FArgs a = I->fa;
  a.t_upd = t;
  a.t_solve = t_solve;
  factor_sample<C, BND>(a, item - l.pre[k], threadIdx.x, lds);
}

// End of a tick: every active instance moves to its next step.
__global__ void advance_kernel(GInst* inst, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const int t = inst[i].t;
    if (t >= 0 && t < inst[i].n_keep) inst[i].t = t + 1;
  }
}

// ------------------------------------------------------- column subsets ----
// Copies sample s's column subset into the work buffer, replacing columns
// outside [0, ldu) by 0 and raising DEV_BADCOLS for those and for repeats
// (a repeated column would make the conditioning matrix singular).
__global__ void colmap_kernel(const int32_t* cols, int32_t* cmap, int32_t* ctl,
                              int k, int ldu) {
  __shared__ uint32_t seen[1024 / 32];
  const int s = blockIdx.x;
  for (int i = threadIdx.x; i < (ldu + 31) / 32; i += blockDim.x) seen[i] = 0u;
  __syncthreads();
  bool bad = false;
  for (int i = threadIdx.x; i < k; i += blockDim.x) {
    int c = cols[(size_t)s * k + i];
    if (c < 0 || c >= ldu) {
      bad = true;
      c = 0;
    }
    const uint32_t bit = 1u << (c & 31);
    if (atomicOr(&seen[c >> 5], bit) & bit) bad = true;
    cmap[(size_t)s * k + i] = c;
  }
  if (bad) atomicOr(&ctl[1], (int)DEV_BADCOLS);
}

// ------------------------------------------------------------ copy-out ----
__global__ void copy_out_kernel(const int32_t* xs, const double* logdet,
                                int32_t* x_out, double* logdet_out, int S,
                                int N, int n_keep) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < (size_t)S * n_keep) {
    const size_t s = i / n_keep, j = i % n_keep;
    x_out[i] = xs[s * N + j];
  }
  if (logdet_out && i < (size_t)S) logdet_out[i] = logdet[i];
}

// ------------------------------------------------------------- density ----
__global__ void density_kernel(const float* ut, double* rho, int L, int L_pad,
                               int N, int Np, int cplx) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= L) return;
  double acc = 0.0;
  for (int k = 0; k < N; ++k) {
    const double v = (double)ut[(size_t)k * L_pad + x];
    acc += v * v;
    if (cplx) {
      const double w = (double)ut[(size_t)(Np + k) * L_pad + x];
      acc += w * w;
    }
  }
  rho[x] = acc;
}

}  // namespace

void launch_init(const Dims& d, const Work& w, int S, hipStream_t st) {
  hipLaunchKernelGGL(init_kernel, dim3(S), dim3(64), 0, st, w.perm, w.logdet,
                     w.occ, w.ctl, w.rec_ctl, w.div, S, d.N, d.L_pad / 32);
}

FArgs make_fargs(const Dims& d, const Work& w, const void* u64, int n_steps,
                 uint64_t seed, uint64_t first) {
  FArgs a;
  a.u64 = u64;
  a.F = w.F;
  a.perm = w.perm;
  a.xs = w.xs;
  a.beta = w.beta;
  a.logdet = w.logdet;
  a.ctl = w.ctl;
  a.gam = static_cast<float*>(w.gam);
  a.gsplit = d.bf16 ? static_cast<uint16_t*>(w.gam) : nullptr;
  a.cmap = w.cmap;
  a.sid = w.sid;
  a.fslot = w.fslot;
  a.wr = w.wr;
  a.cs = w.cs;
  a.occ = w.occ;
  a.counters = w.counters;
  a.L_pad = d.L_pad;
  a.N = d.N;
  a.Np = d.Np;
  a.Kg = d.Kg;
  a.ldu = d.ldu;
  a.t_upd = -1;
  a.t_solve = -1;
  a.n_steps = n_steps;
  a.seed = seed;
  a.first = first;
  return a;
}

template <bool C>
static void launch_factor_t(const Dims& d, const Work& w, const void* u64,
                            int S, int t_upd, int t_solve, int n_steps,
                            uint64_t seed, uint64_t first, hipStream_t st) {
  FArgs a = make_fargs(d, w, u64, n_steps, seed, first);
  a.t_upd = t_upd;
  a.t_solve = t_solve;
  const bool bnd = t_upd >= 0 && t_solve >= 0 && (t_upd % BB) == BB - 1;
  if (bnd) {
    const size_t lds = blk_lds_bytes<C, true>(d.N);
    allow_lds(factor_kernel<C, true>, lds);
    hipLaunchKernelGGL((factor_kernel<C, true>), dim3(S), dim3(64), lds, st, a);
  } else {
    const size_t lds = blk_lds_bytes<C, false>(d.N);
    allow_lds(factor_kernel<C, false>, lds);
    hipLaunchKernelGGL((factor_kernel<C, false>), dim3(S), dim3(64), lds, st, a);
  }
}

template <bool C>
static void launch_drawfactor_t(const Dims& d, const Work& w, const void* u64, int S,
                                int t_upd, int t_solve, int n_steps, uint64_t seed,
                                uint64_t first, double delta, double coef, int row0,
                                hipStream_t st) {
  FArgs a = make_fargs(d, w, u64, n_steps, seed, first);
  a.t_upd = t_upd;
  a.t_solve = t_solve;
  a.fslot = nullptr;
  DArgs g = make_dargs(d, w, S, seed, first, delta, coef, 0);
  g.t = t_upd;
  g.fslot = nullptr;
  g.rec_meta = w.rec_meta;
  g.rec_g = w.rec_g;
  g.rec_occ = w.rec_occ;
  g.rec_cap = w.rec_cap;
  g.row0 = row0;
  const bool bnd = t_solve >= 0 && (t_upd % BB) == BB - 1;
  if (bnd) {
    const size_t lds = blk_lds_bytes<C, true>(d.N);
    allow_lds(drawfactor_kernel<C, true>, lds);
    hipLaunchKernelGGL((drawfactor_kernel<C, true>), dim3(S), dim3(64), lds, st, a, g);
  } else {
    const size_t lds = blk_lds_bytes<C, false>(d.N);
    allow_lds(drawfactor_kernel<C, false>, lds);
    hipLaunchKernelGGL((drawfactor_kernel<C, false>), dim3(S), dim3(64), lds, st, a, g);
  }
}

void launch_drawfactor(const Dims& d, const Work& w, const void* u64, int S, int t_upd,
                       int t_solve, int n_steps, uint64_t seed, uint64_t first, double delta,
                       double coef, int row0, hipStream_t st) {
  if (d.cplx)
    launch_drawfactor_t<true>(d, w, u64, S, t_upd, t_solve, n_steps, seed, first, delta, coef,
                              row0, st);
  else
    launch_drawfactor_t<false>(d, w, u64, S, t_upd, t_solve, n_steps, seed, first, delta, coef,
                               row0, st);
}

void launch_scatter_out(const Dims& d, const Work& w, int n, int n_keep, const int32_t* rows,
                        int32_t* x_out, double* logdet_out, hipStream_t st) {
  const size_t m = (size_t)n * (n_keep > 1 ? n_keep : 1);
  hipLaunchKernelGGL(scatter_out_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st,
                     w.xs, w.logdet, rows, n, d.N, n_keep, x_out, logdet_out);
}

void launch_factor(const Dims& d, const Work& w, const void* u64, int S,
                   int t_upd, int t_solve, int n_steps, uint64_t seed,
                   uint64_t first, hipStream_t st) {
  if (d.cplx)
    launch_factor_t<true>(d, w, u64, S, t_upd, t_solve, n_steps, seed, first, st);
  else
    launch_factor_t<false>(d, w, u64, S, t_upd, t_solve, n_steps, seed, first, st);
}

void launch_colmap(const Dims& d, const Work& w, const int32_t* cols, int S,
                   hipStream_t st) {
  hipLaunchKernelGGL(colmap_kernel, dim3(S), dim3(256), 0, st, cols, w.cmap_buf,
                     w.ctl, d.N, d.ldu);
}

void launch_copy_out(const Dims& d, const Work& w, int S, int n_keep,
                     int32_t* x_out, double* logdet_out, hipStream_t st) {
  const size_t n = (size_t)S * (n_keep > 1 ? n_keep : 1);
  const unsigned blocks = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(copy_out_kernel, dim3(blocks), dim3(256), 0, st, w.xs,
                     w.logdet, x_out, logdet_out, S, d.N, n_keep);
}

void launch_density(const Dims& d, const void* ubulk_t, double* rho,
                    hipStream_t st) {
  hipLaunchKernelGGL(density_kernel, dim3((d.L + 255) / 256), dim3(256), 0, st,
                     static_cast<const float*>(ubulk_t), rho, d.L, d.L_pad, d.N,
                     d.Np, d.cplx);
}

}  // namespace ffsk

namespace ffsk {

template <bool C>
static void launch_factor_group_t(const GInst* inst, const GList& l, int maxN, hipStream_t st) {
  const int grid = l.total;
  const size_t lr = blk_lds_bytes<C, false>(maxN), lb = blk_lds_bytes<C, true>(maxN);
  allow_lds(factor_group_kernel<C, false>, lr);
  hipLaunchKernelGGL((factor_group_kernel<C, false>), dim3(grid), dim3(64), lr, st, inst, l);
  allow_lds(factor_group_kernel<C, true>, lb);
  hipLaunchKernelGGL((factor_group_kernel<C, true>), dim3(grid), dim3(64), lb, st, inst, l);
}

void launch_factor_group(const GInst* inst, const GList& l, bool cplx, int maxN,
                         hipStream_t st) {
  if (l.total == 0) return;
  if (cplx)
    launch_factor_group_t<true>(inst, l, maxN, st);
  else
    launch_factor_group_t<false>(inst, l, maxN, st);
}

void launch_advance(GInst* inst, int n, hipStream_t st) {
  hipLaunchKernelGGL(advance_kernel, dim3((n + 255) / 256), dim3(256), 0, st, inst, n);
}

size_t factor_state_bytes(const Dims& d) {
  return blk_state_elems(d.N) * (d.cplx ? 16 : 8);
}
}  // namespace ffsk
