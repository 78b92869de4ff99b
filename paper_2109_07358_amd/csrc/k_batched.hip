// Batched-path kernels other than the contraction: per-call init, the
// per-step factor kernel (one wavefront per sample), the inverse-CDF draw
// with its near-tie guard, the float64 redraw of guarded draws, copy-out and
// the density hook.
#include "factor.h"
#include "ffs_internal.h"

namespace ffsk {

namespace {

// ---------------------------------------------------------------- init ----
__global__ void init_kernel(int32_t* perm, double* logdet, uint32_t* occ,
                            int32_t* ctl, int S, int N, int nblk) {
  const int s = blockIdx.x;
  if (s >= S) return;
  for (int i = threadIdx.x; i < N; i += blockDim.x) perm[(size_t)s * N + i] = i;
  for (int i = threadIdx.x; i < nblk; i += blockDim.x) occ[(size_t)s * nblk + i] = 0u;
  if (threadIdx.x == 0) {
    logdet[s] = 0.0;
    if (s == 0) ctl[0] = 0;
  }
}

// -------------------------------------------------------------- factor ----
struct FArgs {
  const void* u64;
  void* F;
  int32_t* perm;
  const int32_t* xs;
  void* beta;
  double* logdet;
  int32_t* ctl;
  float* gam;
  int N, Np, Kg, t_upd, t_solve;
  uint64_t seed, first;
};

template <bool C, int TW>
__global__ __launch_bounds__(64) void factor_kernel(FArgs a) {
  using X = Cx<C>;
  using T = typename X::T;
  extern __shared__ __align__(16) char lds[];
  const int s = blockIdx.x;
  const int lane = threadIdx.x;
  if (s == 0 && lane == 0) a.ctl[0] = 0;  // flag count of the coming draw
  FacSample f;
  f.u64 = a.u64;
  f.F = reinterpret_cast<T*>(a.F) + (size_t)s * a.N * a.N;
  f.perm = a.perm + (size_t)s * a.N;
  f.xs = a.xs + (size_t)s * a.N;
  f.beta = reinterpret_cast<T*>(a.beta) + (size_t)s * a.N;
  f.logdet = a.logdet + s;
  f.status = a.ctl + 1;
  f.N = a.N;
  f.seed = a.seed;
  f.sample = a.first + (uint64_t)s;
  T* gl;
  int* pl;
  factor_wave<C, TW>(f, a.t_upd, a.t_solve, lane, lds, &gl, &pl);
  if (a.t_solve < 0) return;
  float* g = a.gam + (size_t)s * a.Kg;
  for (int i = lane; i < a.N; i += 64) {
    const T v = gl[i];
    g[i] = (float)X::re(v);
    if (C) g[a.Np + i] = (float)X::im(v);
  }
}

// ---------------------------------------------------------------- draw ----
struct DArgs {
  const double* bsum;  // [nblk][S_pad]
  const float* wh;     // [S_pad][L_pad]
  int32_t* xs;         // [S_pad][N]
  uint32_t* occ;       // [S_pad][nblk]
  int32_t* ctl;        // [0] flag count, [1] status
  int32_t* flag_list;
  unsigned long long* counters;
  const int32_t* forced;
  int S, S_pad, L_pad, N, t, n_forced;
  double delta;
  uint64_t seed, first;
};

// Inverse CDF over ascending sites: x = first site whose running float64 sum
// F exceeds u*T, T the float64 total.  Running sums are formed from the
// float64 32-site block sums (C_b, fixed order) and, inside the selected
// block, sequentially from its stored float32 weights; the last site of a
// block takes the boundary C_b itself so the two levels agree exactly.  A
// draw is flagged for the float64 redraw when u*T lies within delta*T of an
// end of the selected site's interval (or when the two levels disagree at a
// block end, which can only happen at rounding level).
__global__ __launch_bounds__(256) void draw_kernel(DArgs a) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= a.S) return;
  const int nblk = a.L_pad / 32;
  int32_t* xrow = a.xs + (size_t)s * a.N;
  if (a.t < a.n_forced) {  // teacher forcing (test hook)
    const int x = a.forced[a.t];
    xrow[a.t] = x;
    atomicOr(&a.occ[(size_t)s * nblk + (x >> 5)], 1u << (x & 31));
    return;
  }
  const double* bs = a.bsum + s;
  double T = 0.0;
  for (int b = 0; b < nblk; ++b) T += bs[(size_t)b * a.S_pad];
  const Words wd = philox_block(a.seed, a.first + (uint64_t)s, (uint32_t)a.t);
  const double u = uniform53(wd);
  bool flag = false;
  if (!(T > 0.0) || !isfinite(T)) {
    atomicOr(&a.ctl[1], (int)DEV_NUMERICAL);
    xrow[a.t] = 0;
    return;
  }
  const double target = u * T;
  double C = 0.0, Cn = 0.0;
  int blk = -1;
  for (int b = 0; b < nblk; ++b) {
    Cn = C + bs[(size_t)b * a.S_pad];
    if (Cn > target) {
      blk = b;
      break;
    }
    C = Cn;
  }
  if (blk < 0) {  // u*T at or above the total: last block with mass
    flag = true;
    C = 0.0;
    for (int b = 0; b < nblk; ++b)
      if (bs[(size_t)b * a.S_pad] > 0.0) blk = b;
    for (int b = 0; b < blk; ++b) C += bs[(size_t)b * a.S_pad];
    Cn = C + bs[(size_t)blk * a.S_pad];
  }
  const float* wp = a.wh + (size_t)s * a.L_pad + (size_t)blk * 32;
  float w[32];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const float4 v = reinterpret_cast<const float4*>(wp)[q];
    w[4 * q] = v.x;
    w[4 * q + 1] = v.y;
    w[4 * q + 2] = v.z;
    w[4 * q + 3] = v.w;
  }
  double P = 0.0, prev = C, lo = C, hi = Cn;
  int x = -1, last = -1;
#pragma unroll
  for (int j = 0; j < 32; ++j) {
    const double wj = (double)w[j];
    P += wj;
    const double F = (j == 31) ? Cn : C + P;
    if (wj > 0.0) {
      last = j;
      if (x < 0 && F > target) {
        x = j;
        lo = prev;
        hi = F;
      }
    }
    prev = F;
  }
  if (x < 0) {  // block-end disagreement at rounding level
    flag = true;
    x = last;
    lo = hi = target;
  }
  const double margin = fmin(target - lo, hi - target);
  if (margin < a.delta * T) flag = true;
  const int site = blk * 32 + x;
  xrow[a.t] = site;
  if (flag) {
    const int slot = atomicAdd(&a.ctl[0], 1);
    a.flag_list[slot] = s;
    atomicAdd(&a.counters[0], 1ull);
  } else {
    atomicOr(&a.occ[(size_t)s * nblk + (site >> 5)], 1u << (site & 31));
  }
}

// -------------------------------------------------------------- repair ----
struct RArgs {
  const void* u64t;    // [N][L_pad] column-major float64 / complex128
  const int32_t* perm;
  const void* beta;
  int32_t* xs;
  uint32_t* occ;
  const int32_t* ctl;
  const int32_t* flag_list;
  unsigned long long* counters;
  double* wr;          // [FMAX][L_pad]
  int L_pad, N, t;
  uint64_t seed, first;
};

// Float64 redraw of the flagged draws of step t, one workgroup per flagged
// sample: v(y) = sum_{i<=t} U[y, m_i] g_i with g_t = 1, g_i = -beta_i,
// w = |v|^2 with occupied sites zeroed, running float64 sums in site order
// (256-site chunk sums, then in-chunk), same uniform u as the first draw.
template <bool C>
__global__ __launch_bounds__(256) void repair_kernel(RArgs a) {
  using X = Cx<C>;
  using T = typename X::T;
  __shared__ T gc[1024];
  __shared__ int gm[1024];
  __shared__ double cs[65536 / RCHUNK];
  __shared__ int sel;
  const int tid = threadIdx.x;
  const int count = a.ctl[0];
  const int nblk = a.L_pad / 32;
  const int nch = a.L_pad / RCHUNK;
  const T* U = reinterpret_cast<const T*>(a.u64t);
  double* wr = a.wr + (size_t)blockIdx.x * a.L_pad;
  for (int f = blockIdx.x; f < count; f += gridDim.x) {
    const int s = a.flag_list[f];
    const int32_t* pm = a.perm + (size_t)s * a.N;
    const T* bv = reinterpret_cast<const T*>(a.beta) + (size_t)s * a.N;
    const uint32_t* oc = a.occ + (size_t)s * nblk;
    for (int i = tid; i <= a.t; i += 256) {
      gm[i] = pm[i];
      gc[i] = (i == a.t) ? X::one() : X::neg(bv[i]);
    }
    __syncthreads();
    for (int x0 = 0; x0 < a.L_pad; x0 += 256 * 8) {
      T acc[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) acc[q] = X::zero();
      for (int i = 0; i <= a.t; ++i) {
        const T* col = U + (size_t)gm[i] * a.L_pad;
        const T g = gc[i];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int x = x0 + tid + 256 * q;
          if (x < a.L_pad) acc[q] = X::fma(col[x], g, acc[q]);
        }
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int x = x0 + tid + 256 * q;
        if (x < a.L_pad) {
          const bool occd = (oc[x >> 5] >> (x & 31)) & 1u;
          wr[x] = occd ? 0.0 : X::abs2(acc[q]);
        }
      }
    }
    __syncthreads();
    for (int c = tid; c < nch; c += 256) {
      double sum = 0.0;
      for (int j = 0; j < RCHUNK; ++j) sum += wr[(size_t)c * RCHUNK + j];
      cs[c] = sum;
    }
    __syncthreads();
    if (tid == 0) {
      double T64 = 0.0;
      for (int c = 0; c < nch; ++c) T64 += cs[c];
      const Words wd = philox_block(a.seed, a.first + (uint64_t)s, (uint32_t)a.t);
      const double target = uniform53(wd) * T64;
      double Cc = 0.0, Cn = 0.0;
      int ch = -1;
      for (int c = 0; c < nch; ++c) {
        Cn = Cc + cs[c];
        if (Cn > target) {
          ch = c;
          break;
        }
        Cc = Cn;
      }
      if (ch < 0) {
        Cc = 0.0;
        for (int c = 0; c < nch; ++c)
          if (cs[c] > 0.0) ch = c;
        for (int c = 0; c < ch; ++c) Cc += cs[c];
        if (ch >= 0) Cn = Cc + cs[ch];
      }
      if (ch < 0) {  // no float64 mass at all: report, keep the first draw
        atomicOr((int*)&a.ctl[1], (int)DEV_NUMERICAL);
        sel = a.xs[(size_t)s * a.N + a.t];
      } else {
        double Pp = 0.0;
        int x = -1, last = -1;
        for (int j = 0; j < RCHUNK; ++j) {
          const double wj = wr[(size_t)ch * RCHUNK + j];
          Pp += wj;
          const double F = (j == RCHUNK - 1) ? Cn : Cc + Pp;
          if (wj > 0.0) {
            last = j;
            if (x < 0 && F > target) x = j;
          }
        }
        if (x < 0) x = last;
        sel = ch * RCHUNK + x;
      }
    }
    __syncthreads();
    if (tid == 0) {
      const int site = sel;
      int32_t* xrow = a.xs + (size_t)s * a.N;
      if (xrow[a.t] != site) atomicAdd(&a.counters[1], 1ull);
      xrow[a.t] = site;
      atomicOr(&a.occ[(size_t)s * nblk + (site >> 5)], 1u << (site & 31));
    }
    __syncthreads();
  }
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
                     w.occ, w.ctl, S, d.N, d.L_pad / 32);
}

template <bool C, int TW>
static void launch_factor_t(const Dims& d, const Work& w, const void* u64,
                            int S, int t_upd, int t_solve, uint64_t seed,
                            uint64_t first, hipStream_t st) {
  FArgs a;
  a.u64 = u64;
  a.F = w.F;
  a.perm = w.perm;
  a.xs = w.xs;
  a.beta = w.beta;
  a.logdet = w.logdet;
  a.ctl = w.ctl;
  a.gam = static_cast<float*>(w.gam);
  a.N = d.N;
  a.Np = d.Np;
  a.Kg = d.Kg;
  a.t_upd = t_upd;
  a.t_solve = t_solve;
  a.seed = seed;
  a.first = first;
  const size_t lds = factor_lds_bytes<C>(d.N);
  allow_lds(factor_kernel<C, TW>, lds);
  hipLaunchKernelGGL((factor_kernel<C, TW>), dim3(S), dim3(64), lds, st, a);
}

void launch_factor(const Dims& d, const Work& w, const void* u64, int S,
                   int t_upd, int t_solve, uint64_t seed, uint64_t first,
                   hipStream_t st) {
  if (d.cplx)
    launch_factor_t<true, 16>(d, w, u64, S, t_upd, t_solve, seed, first, st);
  else
    launch_factor_t<false, 32>(d, w, u64, S, t_upd, t_solve, seed, first, st);
}

void launch_draw(const Dims& d, const Work& w, int S, int t, uint64_t seed,
                 uint64_t first, double delta, int n_forced, hipStream_t st) {
  DArgs a;
  a.bsum = w.bsum;
  a.wh = static_cast<const float*>(w.wh);
  a.xs = w.xs;
  a.occ = w.occ;
  a.ctl = w.ctl;
  a.flag_list = w.flag_list;
  a.counters = w.counters;
  a.forced = w.forced;
  a.S = S;
  a.S_pad = w.S_pad;
  a.L_pad = d.L_pad;
  a.N = d.N;
  a.t = t;
  a.n_forced = n_forced;
  a.delta = delta;
  a.seed = seed;
  a.first = first;
  hipLaunchKernelGGL(draw_kernel, dim3((S + 255) / 256), dim3(256), 0, st, a);
}

void launch_repair(const Dims& d, const Work& w, const void* u64t, int S,
                   int t, uint64_t seed, uint64_t first, hipStream_t st) {
  RArgs a;
  a.u64t = u64t;
  a.perm = w.perm;
  a.beta = w.beta;
  a.xs = w.xs;
  a.occ = w.occ;
  a.ctl = w.ctl;
  a.flag_list = w.flag_list;
  a.counters = w.counters;
  a.wr = w.wr;
  a.L_pad = d.L_pad;
  a.N = d.N;
  a.t = t;
  a.seed = seed;
  a.first = first;
  const int grid = S < FMAX ? S : FMAX;
  if (d.cplx)
    hipLaunchKernelGGL(repair_kernel<true>, dim3(grid), dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL(repair_kernel<false>, dim3(grid), dim3(256), 0, st, a);
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
