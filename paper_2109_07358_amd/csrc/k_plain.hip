// Plain path: one launch draws one sample, all steps fused in a single
// workgroup -- the paper's own single-sample regime (Eq. (2) with the
// geometric conditionals of Eq. (3), 2Nk + 2Lk operations at step k).
//
// Per step t: wavefront 0 runs the float64 factor update/solve (factor.h);
// then all 256 threads evaluate v(y) = sum_{i<=t} U[y, m_i] g_i over every
// site y with only the t+1 non-zero coefficients (the true 2Lk work, reading
// U column-major so each column read is coalesced), square, mask, and store
// the weights; 32-site float64 block sums give the inverse-CDF scan.  With
// float32 bulk a draw within delta*T of a boundary is redone from float64
// weights (same rule as the batched path).
#include "factor.h"
#include "ffs_internal.h"

namespace ffsk {

namespace {

struct PArgs {
  const void* u64;     // [L][N] row-major float64/complex128
  const void* u64t;    // [N][L_pad] column-major float64/complex128
  const float* u32t;   // [K][L_pad] bulk float32 (complex: Ur rows, Ui rows)
  void* F;             // scratch [N][N]
  void* beta;          // scratch [N]
  int32_t* perm;       // scratch [N]
  int32_t* xs;         // scratch [N]
  void* wq;            // scratch [L_pad] bulk weights (float or double)
  double* wr;          // scratch [L_pad] float64 weights
  double* ld;          // scratch [1]
  int32_t* x_out;      // [n_keep]
  double* logdet_out;  // nullable
  int32_t* ctl;        // [1] status
  unsigned long long* counters;
  int L, L_pad, N, Np, n_keep;
  double delta;
  uint64_t seed, sample;
};

template <bool C, bool B64, int TW>
__global__ __launch_bounds__(256) void plain_kernel(PArgs a) {
  using X = Cx<C>;
  using T = typename X::T;
  extern __shared__ __align__(16) char lds[];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int N = a.N;
  const int nblk = a.L_pad / 32;
  const int nch = a.L_pad / RCHUNK;
  char* p = lds;
  void* flds = p;
  p += (factor_lds_bytes<C>(N) + 15) / 16 * 16;
  T* gc64 = reinterpret_cast<T*>(p);
  p += (size_t)N * sizeof(T);
  int* gm = reinterpret_cast<int*>(p);
  p += (size_t)N * 4;
  uint32_t* occ = reinterpret_cast<uint32_t*>(p);
  p += (size_t)nblk * 4;
  p = lds + ((p - lds) + 7) / 8 * 8;
  double* bsl = reinterpret_cast<double*>(p);
  p += (size_t)nblk * 8;
  double* csl = reinterpret_cast<double*>(p);
  __shared__ int sel_x;
  __shared__ int need_repair;

  for (int i = tid; i < nblk; i += 256) occ[i] = 0u;
  for (int i = tid; i < N; i += 256) a.perm[i] = i;
  if (tid == 0) *a.ld = 0.0;
  __syncthreads();

  FacSample f;
  f.u64 = a.u64;
  f.F = a.F;
  f.perm = a.perm;
  f.xs = a.xs;
  f.beta = a.beta;
  f.logdet = a.ld;
  f.status = a.ctl + 1;
  f.N = N;
  f.seed = a.seed;
  f.sample = a.sample;

  const T* U64t = reinterpret_cast<const T*>(a.u64t);
  for (int t = 0; t <= a.n_keep; ++t) {
    const int t_solve = (t < a.n_keep) ? t : -1;
    if (wave == 0) {
      T* gl;
      int* pl;
      factor_wave<C, TW>(f, t - 1, t_solve, lane, flds, &gl, &pl);
      if (t_solve >= 0) {
        // coefficient list: g_i = -beta_i (i < t), g_t = 1, on columns m_i
        const T* zl = reinterpret_cast<const T*>(flds) + 2 * N;
        for (int i = lane; i <= t; i += 64) {
          gm[i] = pl[i];
          gc64[i] = (i == t) ? X::one() : X::neg(zl[i]);
        }
      }
    }
    __syncthreads();
    if (t_solve < 0) break;

    // ---- bulk weights over all sites ---------------------------------------
    for (int x0 = 0; x0 < a.L_pad; x0 += 256 * 4) {
      if (B64) {
        T acc[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] = X::zero();
        for (int i = 0; i <= t; ++i) {
          const T* col = U64t + (size_t)gm[i] * a.L_pad;
          const T g = gc64[i];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int x = x0 + tid + 256 * q;
            if (x < a.L_pad) acc[q] = X::fma(col[x], g, acc[q]);
          }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int x = x0 + tid + 256 * q;
          if (x < a.L_pad) {
            const bool o = (occ[x >> 5] >> (x & 31)) & 1u;
            reinterpret_cast<double*>(a.wq)[x] = o ? 0.0 : X::abs2(acc[q]);
          }
        }
      } else {
        float ar[4] = {0.f, 0.f, 0.f, 0.f}, ai[4] = {0.f, 0.f, 0.f, 0.f};
        for (int i = 0; i <= t; ++i) {
          const int m = gm[i];
          const T g = gc64[i];
          const float gr = (float)X::re(g), gi = (float)X::im(g);
          const float* cr = a.u32t + (size_t)m * a.L_pad;
          const float* ci = a.u32t + (size_t)(a.Np + m) * a.L_pad;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int x = x0 + tid + 256 * q;
            if (x < a.L_pad) {
              const float ur = cr[x];
              if (C) {
                const float ui = ci[x];
                ar[q] = fmaf(ur, gr, fmaf(-ui, gi, ar[q]));
                ai[q] = fmaf(ur, gi, fmaf(ui, gr, ai[q]));
              } else {
                ar[q] = fmaf(ur, gr, ar[q]);
              }
            }
          }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int x = x0 + tid + 256 * q;
          if (x < a.L_pad) {
            const bool o = (occ[x >> 5] >> (x & 31)) & 1u;
            const float w = C ? ar[q] * ar[q] + ai[q] * ai[q] : ar[q] * ar[q];
            reinterpret_cast<float*>(a.wq)[x] = o ? 0.0f : w;
          }
        }
      }
    }
    __syncthreads();
    for (int b = tid; b < nblk; b += 256) {
      double sum = 0.0;
      for (int j = 0; j < 32; ++j) {
        const int x = 32 * b + j;
        sum += B64 ? reinterpret_cast<const double*>(a.wq)[x]
                   : (double)reinterpret_cast<const float*>(a.wq)[x];
      }
      bsl[b] = sum;
    }
    __syncthreads();
    if (tid == 0) {
      double T = 0.0;
      for (int b = 0; b < nblk; ++b) T += bsl[b];
      const double target = uniform53(philox_block(a.seed, a.sample, (uint32_t)t)) * T;
      bool flag = false;
      int site = 0;
      if (!(T > 0.0) || !isfinite(T)) {
        atomicOr(&a.ctl[1], (int)DEV_NUMERICAL);
      } else {
        double Cc = 0.0, Cn = 0.0;
        int blk = -1;
        for (int b = 0; b < nblk; ++b) {
          Cn = Cc + bsl[b];
          if (Cn > target) {
            blk = b;
            break;
          }
          Cc = Cn;
        }
        if (blk < 0) {
          flag = true;
          Cc = 0.0;
          for (int b = 0; b < nblk; ++b)
            if (bsl[b] > 0.0) blk = b;
          for (int b = 0; b < blk; ++b) Cc += bsl[b];
          Cn = Cc + bsl[blk];
        }
        double P = 0.0, prev = Cc, lo = Cc, hi = Cn;
        int x = -1, last = -1;
        for (int j = 0; j < 32; ++j) {
          const int xx = 32 * blk + j;
          const double wj = B64 ? reinterpret_cast<const double*>(a.wq)[xx]
                                : (double)reinterpret_cast<const float*>(a.wq)[xx];
          P += wj;
          const double F = (j == 31) ? Cn : Cc + P;
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
        if (x < 0) {
          flag = true;
          x = last;
          lo = hi = target;
        }
        if (fmin(target - lo, hi - target) < a.delta * T) flag = true;
        site = 32 * blk + x;
      }
      sel_x = site;
      need_repair = flag ? 1 : 0;
      if (flag) atomicAdd(&a.counters[0], 1ull);
    }
    __syncthreads();

    if (need_repair) {  // float64 redraw, same uniform
      for (int x0 = 0; x0 < a.L_pad; x0 += 256 * 4) {
        T acc[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] = X::zero();
        for (int i = 0; i <= t; ++i) {
          const T* col = U64t + (size_t)gm[i] * a.L_pad;
          const T g = gc64[i];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int x = x0 + tid + 256 * q;
            if (x < a.L_pad) acc[q] = X::fma(col[x], g, acc[q]);
          }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int x = x0 + tid + 256 * q;
          if (x < a.L_pad) {
            const bool o = (occ[x >> 5] >> (x & 31)) & 1u;
            a.wr[x] = o ? 0.0 : X::abs2(acc[q]);
          }
        }
      }
      __syncthreads();
      for (int c = tid; c < nch; c += 256) {
        double sum = 0.0;
        for (int j = 0; j < RCHUNK; ++j) sum += a.wr[(size_t)c * RCHUNK + j];
        csl[c] = sum;
      }
      __syncthreads();
      if (tid == 0) {
        double T64 = 0.0;
        for (int c = 0; c < nch; ++c) T64 += csl[c];
        const double target = uniform53(philox_block(a.seed, a.sample, (uint32_t)t)) * T64;
        double Cc = 0.0, Cn = 0.0;
        int ch = -1;
        for (int c = 0; c < nch; ++c) {
          Cn = Cc + csl[c];
          if (Cn > target) {
            ch = c;
            break;
          }
          Cc = Cn;
        }
        if (ch < 0) {
          Cc = 0.0;
          for (int c = 0; c < nch; ++c)
            if (csl[c] > 0.0) ch = c;
          for (int c = 0; c < ch; ++c) Cc += csl[c];
          if (ch >= 0) Cn = Cc + csl[ch];
        }
        if (ch < 0) {
          atomicOr(&a.ctl[1], (int)DEV_NUMERICAL);
        } else {
          double P = 0.0;
          int x = -1, last = -1;
          for (int j = 0; j < RCHUNK; ++j) {
            const double wj = a.wr[(size_t)ch * RCHUNK + j];
            P += wj;
            const double F = (j == RCHUNK - 1) ? Cn : Cc + P;
            if (wj > 0.0) {
              last = j;
              if (x < 0 && F > target) x = j;
            }
          }
          if (x < 0) x = last;
          const int site = ch * RCHUNK + x;
          if (site != sel_x) atomicAdd(&a.counters[1], 1ull);
          sel_x = site;
        }
      }
      __syncthreads();
    }
    if (tid == 0) {
      const int site = sel_x;
      a.xs[t] = site;
      a.x_out[t] = site;
      occ[site >> 5] |= 1u << (site & 31);
    }
    __syncthreads();
  }
  if (tid == 0 && a.logdet_out) *a.logdet_out = *a.ld;
}

template <bool C>
size_t plain_lds(int N, int L_pad) {
  const int nblk = L_pad / 32, nch = L_pad / RCHUNK;
  size_t b = (factor_lds_bytes<C>(N) + 15) / 16 * 16;
  b += (size_t)N * (C ? 16 : 8) + (size_t)N * 4 + (size_t)nblk * 4;
  b = (b + 7) / 8 * 8;
  b += (size_t)nblk * 8 + (size_t)nch * 8;
  return b;
}

}  // namespace

size_t plain_scratch_bytes(const Dims& d) {
  const size_t es = d.cplx ? 16 : 8;
  size_t b = (size_t)d.N * d.N * es;  // F
  b += (size_t)d.N * es;              // beta
  b += (size_t)d.N * 4 * 2;           // perm, xs
  b += (size_t)d.L_pad * 8;           // wq
  b += (size_t)d.L_pad * 8;           // wr
  b += 64;                            // ld
  return (b + 255) / 256 * 256 + 1024;
}

void launch_plain(const Dims& d, const void* u64, const void* u64t,
                  const void* ubulk_t, uint64_t seed, uint64_t sample,
                  int n_keep, double delta, void* scratch, int32_t* x_out,
                  double* logdet_out, int32_t* ctl,
                  unsigned long long* counters, hipStream_t st) {
  const size_t es = d.cplx ? 16 : 8;
  char* p = static_cast<char*>(scratch);
  auto take = [&](size_t n) {
    char* r = p;
    p += (n + 255) / 256 * 256;
    return r;
  };
  PArgs a;
  a.u64 = u64;
  a.u64t = u64t;
  a.u32t = static_cast<const float*>(ubulk_t);
  a.F = take((size_t)d.N * d.N * es);
  a.beta = take((size_t)d.N * es);
  a.perm = reinterpret_cast<int32_t*>(take((size_t)d.N * 4));
  a.xs = reinterpret_cast<int32_t*>(take((size_t)d.N * 4));
  a.wq = take((size_t)d.L_pad * 8);
  a.wr = reinterpret_cast<double*>(take((size_t)d.L_pad * 8));
  a.ld = reinterpret_cast<double*>(take(64));
  a.x_out = x_out;
  a.logdet_out = logdet_out;
  a.ctl = ctl;
  a.counters = counters;
  a.L = d.L;
  a.L_pad = d.L_pad;
  a.N = d.N;
  a.Np = d.Np;
  a.n_keep = n_keep;
  a.delta = d.bulk64 ? 0.0 : delta;
  a.seed = seed;
  a.sample = sample;
  if (d.cplx) {
    const size_t lds = plain_lds<true>(d.N, d.L_pad);
    if (d.bulk64)
      {
        allow_lds(plain_kernel<true, true, 16>, lds);
        hipLaunchKernelGGL((plain_kernel<true, true, 16>), dim3(1), dim3(256), lds, st, a);
      }
    else
      {
        allow_lds(plain_kernel<true, false, 16>, lds);
        hipLaunchKernelGGL((plain_kernel<true, false, 16>), dim3(1), dim3(256), lds, st, a);
      }
  } else {
    const size_t lds = plain_lds<false>(d.N, d.L_pad);
    if (d.bulk64)
      {
        allow_lds(plain_kernel<false, true, 32>, lds);
        hipLaunchKernelGGL((plain_kernel<false, true, 32>), dim3(1), dim3(256), lds, st, a);
      }
    else
      {
        allow_lds(plain_kernel<false, false, 32>, lds);
        hipLaunchKernelGGL((plain_kernel<false, false, 32>), dim3(1), dim3(256), lds, st, a);
      }
  }
}

}  // namespace ffsk
