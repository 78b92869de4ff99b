// Plain path: one launch draws one sample, all steps fused in a single
// workgroup -- the paper's own single-sample regime (Eq. (2) with the
// geometric conditionals of Eq. (3), 2Nk + 2Lk operations at step k).
//
// Per step t: the whole workgroup runs the float64 factor update/solve
// (factor_wg.h); then all 512 threads evaluate v(y) = sum_{i<=t} U[y, m_i] g_i over every
// site y with only the t+1 non-zero coefficients (the true 2Lk work).  U is
// read column-major, four consecutive sites per thread and several columns
// in flight, so the step streams U[:, m_<=t] at the bandwidth of the one CU
// the launch occupies.  Weights are squared and masked in registers, stored,
// and summed in float64 per aligned 32-site block by 8-lane shuffles;
// wavefront 0 then runs the inverse-CDF search over block sums and within
// the chosen block.  With float32 bulk a draw within delta*T of a boundary
// is redone from float64 weights (same rule as the batched path).
#include "factor_wg.h"
#include "ffs_internal.h"

#include <type_traits>

namespace ffsk {

namespace {

constexpr int PT = 512;  // threads per workgroup (8 wavefronts)
constexpr int SPT = 4;   // consecutive sites per thread per pass

struct PArgs {
  const void* u64;     // [L][N] row-major float64/complex128
  const void* u64t;    // [N][L_pad] column-major float64/complex128
  const float* u32t;   // [K][L_pad] bulk float32 (complex: Ur rows, Ui rows)
  void* F;             // scratch 4 x [N][N]: Li col-major, Li row-major, P col-, P row-major
  int32_t* xs;         // scratch [N]
  void* wq;            // scratch [L_pad] bulk weights (float or double)
  double* wr;          // scratch [L_pad] float64 weights of a redraw
  double* ld;          // scratch [1]
  int32_t* x_out;      // [n_keep]
  double* logdet_out;  // nullable
  int32_t* ctl;        // [1] status
  unsigned long long* counters;
  int L, L_pad, N, Np, n_keep;
  double delta, coef;  // guard threshold max(delta * T, coef * sqrt(sum_b B_b^2))
  uint64_t seed, sample;
};

// ---- wavefront inverse-CDF search ------------------------------------------
// Values val(0..n-1) >= 0 in site order are split into 64 lane chunks of q
// consecutive values.  chunk_ends returns, per lane, the cumulative value at
// the end of its chunk (base + inclusive lane prefix of the chunk sums, a
// fixed Hillis-Steele order).  With use_end the last chunk ends exactly at
// `end`, the boundary an enclosing level already fixed, so that nested
// levels agree on where the range stops.
template <class Get>
__device__ inline double chunk_ends(Get val, int n, int q, double base,
                                    bool use_end, double end, int lane) {
  const int b0 = lane * q, b1 = min(b0 + q, n);
  double s = 0.0;
  for (int i = b0; i < b1; ++i) s += val(i);
  double p = s;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const double o = __shfl_up(p, d, 64);
    if (lane >= d) p = o + p;
  }
  double E = base + p;
  if (use_end && lane >= (n - 1) / q) E = end;
  return E;
}

struct Hit {
  int i;          // index of the drawn value, -1 if the search found none
  double lo, hi;  // cumulative values before and after it
};

// First i with val(i) > 0 whose cumulative value after it exceeds target.
// The last value of each chunk takes the chunk end from chunk_ends.  Every
// lane returns the same result.
template <class Get>
__device__ inline Hit pick(Get val, int n, int q, double base, double E,
                           double target, int lane) {
  const unsigned long long m = __ballot(lane * q < n && E > target);
  Hit h{-1, 0.0, 0.0};
  if (m == 0ull) return h;
  const int ls = __ffsll((long long)m) - 1;
  const double start = __shfl_up(E, 1, 64);
  if (lane == ls) {
    double F = (ls == 0) ? base : start;
    const int c0 = ls * q, c1 = min(c0 + q, n);
    for (int i = c0; i < c1; ++i) {
      const double v = val(i);
      const double Fn = (i == c1 - 1) ? E : F + v;
      if (v > 0.0 && Fn > target) {
        h.i = i;
        h.lo = F;
        h.hi = Fn;
        break;
      }
      F = Fn;
    }
  }
  h.i = __shfl(h.i, ls, 64);
  h.lo = __shfl(h.lo, ls, 64);
  h.hi = __shfl(h.hi, ls, 64);
  return h;
}

// Largest i with val(i) > 0, -1 if none (fallback when rounding leaves the
// search without a crossing).
template <class Get>
__device__ inline int last_positive(Get val, int n, int lane) {
  int best = -1;
  for (int i = lane; i < n; i += 64)
    if (val(i) > 0.0) best = i;
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) best = max(best, __shfl_xor(best, d, 64));
  return best;
}

// Inverse-CDF draw over the L_pad sites: block sums bsl[nblk], per-site
// weights val(x).  Returns the site and whether the draw must be redone in
// float64 (no clean crossing, or margin below the guard threshold
// max(delta * T, coef * sqrt(sum_b B_b^2)), the same rule as the batched
// draw).
template <class Get>
__device__ inline int draw_site(Get val, const double* bsl, int nblk,
                                double u, double delta, double coef, bool* flag,
                                bool* bad, int lane) {
  *flag = false;
  *bad = false;
  auto bval = [&](int i) { return bsl[i]; };
  const int qb = (nblk + 63) / 64;
  const double E = chunk_ends(bval, nblk, qb, 0.0, false, 0.0, lane);
  const double T = __shfl(E, 63, 64);
  if (!(T > 0.0) || !isfinite(T)) {
    *bad = true;
    return 0;
  }
  const double target = u * T;
  const Hit hb = pick(bval, nblk, qb, 0.0, E, target, lane);
  int blk = hb.i;
  if (blk < 0) {
    *flag = true;
    blk = last_positive(bval, nblk, lane);
    if (blk < 0) {
      *bad = true;
      return 0;
    }
    auto wl = [&](int j) { return val(32 * blk + j); };
    const int j = last_positive(wl, 32, lane);
    return 32 * blk + (j < 0 ? 0 : j);
  }
  auto wv = [&](int j) { return val(32 * blk + j); };
  const double E2 = chunk_ends(wv, 32, 1, hb.lo, true, hb.hi, lane);
  const Hit hs = pick(wv, 32, 1, hb.lo, E2, target, lane);
  if (hs.i < 0) {
    *flag = true;
    const int j = last_positive(wv, 32, lane);
    return 32 * blk + (j < 0 ? 0 : j);
  }
  double p2 = 0.0;
  for (int i = lane; i < nblk; i += 64) p2 += bsl[i] * bsl[i];
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) p2 += __shfl_xor(p2, o, 64);
  if (fmin(target - hs.lo, hs.hi - target) < fmax(delta * T, coef * sqrt(p2))) *flag = true;
  return 32 * blk + hs.i;
}

// ---- gathered GEMV: weights of sites x0..x0+3 ------------------------------
// v(y) = sum_{i<=t} U[y, gm[i]] g_i in a fixed sequential order over i;
// UR columns are loaded before they are used.
template <bool C, bool B64>
struct Site4;

template <>
struct Site4<false, false> {  // float32 real
  static constexpr int UR = 16;
  __device__ static void run(const PArgs& a, int x0, int t, const int* gm,
                             const float* gcf, const double*, double (&w)[4]) {
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    const float* base = a.u32t + x0;
    int i = 0;
    for (; i + UR <= t + 1; i += UR) {
      float4 u[UR];
#pragma unroll
      for (int k = 0; k < UR; ++k)
        u[k] = *reinterpret_cast<const float4*>(base + (size_t)gm[i + k] * a.L_pad);
#pragma unroll
      for (int k = 0; k < UR; ++k) {
        const float g = gcf[i + k];
        acc.x = fmaf(u[k].x, g, acc.x);
        acc.y = fmaf(u[k].y, g, acc.y);
        acc.z = fmaf(u[k].z, g, acc.z);
        acc.w = fmaf(u[k].w, g, acc.w);
      }
    }
    for (; i <= t; ++i) {
      const float4 u = *reinterpret_cast<const float4*>(base + (size_t)gm[i] * a.L_pad);
      const float g = gcf[i];
      acc.x = fmaf(u.x, g, acc.x);
      acc.y = fmaf(u.y, g, acc.y);
      acc.z = fmaf(u.z, g, acc.z);
      acc.w = fmaf(u.w, g, acc.w);
    }
    w[0] = acc.x * acc.x;
    w[1] = acc.y * acc.y;
    w[2] = acc.z * acc.z;
    w[3] = acc.w * acc.w;
  }
};

template <>
struct Site4<true, false> {  // float32 complex (Ur rows, then Ui rows)
  static constexpr int UR = 8;
  __device__ static void run(const PArgs& a, int x0, int t, const int* gm,
                             const float* gcf, const double2*, double (&w)[4]) {
    float ar[4] = {0.f, 0.f, 0.f, 0.f}, ai[4] = {0.f, 0.f, 0.f, 0.f};
    const float* base = a.u32t + x0;
    const size_t im_off = (size_t)a.Np * a.L_pad;
    auto step = [&](const float4& ur4, const float4& ui4, float gr, float gi) {
      const float ur[4] = {ur4.x, ur4.y, ur4.z, ur4.w};
      const float ui[4] = {ui4.x, ui4.y, ui4.z, ui4.w};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        ar[q] = fmaf(ur[q], gr, fmaf(-ui[q], gi, ar[q]));
        ai[q] = fmaf(ur[q], gi, fmaf(ui[q], gr, ai[q]));
      }
    };
    int i = 0;
    for (; i + UR <= t + 1; i += UR) {
      float4 ur[UR], ui[UR];
#pragma unroll
      for (int k = 0; k < UR; ++k) {
        const float* col = base + (size_t)gm[i + k] * a.L_pad;
        ur[k] = *reinterpret_cast<const float4*>(col);
        ui[k] = *reinterpret_cast<const float4*>(col + im_off);
      }
#pragma unroll
      for (int k = 0; k < UR; ++k) step(ur[k], ui[k], gcf[2 * (i + k)], gcf[2 * (i + k) + 1]);
    }
    for (; i <= t; ++i) {
      const float* col = base + (size_t)gm[i] * a.L_pad;
      step(*reinterpret_cast<const float4*>(col),
           *reinterpret_cast<const float4*>(col + im_off), gcf[2 * i], gcf[2 * i + 1]);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) w[q] = ar[q] * ar[q] + ai[q] * ai[q];
  }
};

template <>
struct Site4<false, true> {  // float64 real
  static constexpr int UR = 8;
  __device__ static void run(const PArgs& a, int x0, int t, const int* gm,
                             const float*, const double* g64, double (&w)[4]) {
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const double* base = reinterpret_cast<const double*>(a.u64t) + x0;
    auto step = [&](const double2& lo, const double2& hi, double g) {
      acc[0] = fma(lo.x, g, acc[0]);
      acc[1] = fma(lo.y, g, acc[1]);
      acc[2] = fma(hi.x, g, acc[2]);
      acc[3] = fma(hi.y, g, acc[3]);
    };
    int i = 0;
    for (; i + UR <= t + 1; i += UR) {
      double2 lo[UR], hi[UR];
#pragma unroll
      for (int k = 0; k < UR; ++k) {
        const double* col = base + (size_t)gm[i + k] * a.L_pad;
        lo[k] = *reinterpret_cast<const double2*>(col);
        hi[k] = *reinterpret_cast<const double2*>(col + 2);
      }
#pragma unroll
      for (int k = 0; k < UR; ++k) step(lo[k], hi[k], g64[i + k]);
    }
    for (; i <= t; ++i) {
      const double* col = base + (size_t)gm[i] * a.L_pad;
      step(*reinterpret_cast<const double2*>(col), *reinterpret_cast<const double2*>(col + 2),
           g64[i]);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) w[q] = acc[q] * acc[q];
  }
};

template <>
struct Site4<true, true> {  // complex128
  static constexpr int UR = 4;
  __device__ static void run(const PArgs& a, int x0, int t, const int* gm,
                             const float*, const double2* g64, double (&w)[4]) {
    using X = Cx<true>;
    double2 acc[4] = {X::zero(), X::zero(), X::zero(), X::zero()};
    const double2* base = reinterpret_cast<const double2*>(a.u64t) + x0;
    int i = 0;
    for (; i + UR <= t + 1; i += UR) {
      double2 u[UR][4];
#pragma unroll
      for (int k = 0; k < UR; ++k) {
        const double2* col = base + (size_t)gm[i + k] * a.L_pad;
#pragma unroll
        for (int q = 0; q < 4; ++q) u[k][q] = col[q];
      }
#pragma unroll
      for (int k = 0; k < UR; ++k) {
        const double2 g = g64[i + k];
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] = X::fma(u[k][q], g, acc[q]);
      }
    }
    for (; i <= t; ++i) {
      const double2* col = base + (size_t)gm[i] * a.L_pad;
      const double2 g = g64[i];
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] = X::fma(col[q], g, acc[q]);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) w[q] = X::abs2(acc[q]);
  }
};

// Weights of every site (masked by occupancy) into dst, float64 sums of each
// aligned 32-site block (8 lanes) into bsl.  PT*SPT sites per pass; L_pad is
// a multiple of 256, so each wavefront's 256 sites are all in or all out.
template <bool C, bool B64, typename W>
__device__ inline void all_weights(const PArgs& a, int t, const int* gm,
                                   const float* gcf,
                                   const typename Cx<C>::T* g64,
                                   const uint32_t* occ, W* dst, double* bsl,
                                   int tid) {
  for (int x0 = SPT * tid; x0 < a.L_pad; x0 += SPT * PT) {
    double w[4];
    Site4<C, B64>::run(a, x0, t, gm, gcf, g64, w);
    const uint32_t ow = occ[x0 >> 5] >> (x0 & 31);
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if ((ow >> q) & 1u) w[q] = 0.0;
    if (sizeof(W) == 4) {
      *reinterpret_cast<float4*>(dst + x0) =
          make_float4((float)w[0], (float)w[1], (float)w[2], (float)w[3]);
    } else {
      *reinterpret_cast<double2*>(dst + x0) = make_double2(w[0], w[1]);
      *reinterpret_cast<double2*>(dst + x0 + 2) = make_double2(w[2], w[3]);
    }
    double part = ((w[0] + w[1]) + w[2]) + w[3];
    part += __shfl_xor(part, 1, 64);
    part += __shfl_xor(part, 2, 64);
    part += __shfl_xor(part, 4, 64);
    if ((tid & 7) == 0) bsl[x0 >> 5] = part;
  }
}

template <bool C, bool B64>
__global__ __launch_bounds__(PT) void plain_kernel(PArgs a) {
  using X = Cx<C>;
  using T = typename X::T;
  using WT = typename std::conditional<B64, double, float>::type;
  extern __shared__ __align__(16) char lds[];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int N = a.N;
  const int nblk = a.L_pad / 32;
  char* p = lds;
  const WgLds<C> wl(p, N);
  p += (wg_lds_bytes<C>(N) + 15) / 16 * 16;
  uint32_t* occ = reinterpret_cast<uint32_t*>(p);
  p += (size_t)nblk * 4;
  p = lds + ((p - lds) + 7) / 8 * 8;
  double* bsl = reinterpret_cast<double*>(p);
  // the Gamma coefficient lists reuse factor vectors that are free between
  // two factor steps: column order = pl, float64 coefficients in ll, float32
  // coefficients in gg
  const int* gm = wl.pl;
  T* gc64 = wl.ll;
  float* gcf = reinterpret_cast<float*>(wl.gg);
  __shared__ int sel_x;
  __shared__ int need_repair;

  for (int i = tid; i < nblk; i += PT) occ[i] = 0u;
  for (int i = tid; i < N; i += PT) wl.pl[i] = i;
  if (tid == 0) *a.ld = 0.0;
  __syncthreads();

  WgState<C> f;
  const size_t NN = (size_t)N * N;
  f.u64 = reinterpret_cast<const T*>(a.u64);
  f.LiC = reinterpret_cast<T*>(a.F);
  f.LiR = f.LiC + NN;
  f.PC = f.LiR + NN;
  f.PR = f.PC + NN;
  f.xs = a.xs;
  f.logdet = a.ld;
  f.status = a.ctl + 1;
  f.N = N;
  f.seed = a.seed;
  f.sample = a.sample;
  WT* wq = reinterpret_cast<WT*>(a.wq);
  for (int t = 0; t <= a.n_keep; ++t) {
    const int t_solve = (t < a.n_keep) ? t : -1;
    factor_wg<C>(f, t - 1, t_solve, wl, tid, PT);
    if (t_solve < 0) break;
    // coefficient list: g_i = -beta_i (i < t), g_t = 1, on columns m_i
    for (int i = tid; i <= t; i += PT) {
      const T g = (i == t) ? X::one() : X::neg(wl.bet[i]);
      gc64[i] = g;
      gcf[C ? 2 * i : i] = (float)X::re(g);
      if (C) gcf[2 * i + 1] = (float)X::im(g);
    }
    __syncthreads();

    all_weights<C, B64>(a, t, gm, gcf, gc64, occ, wq, bsl, tid);
    __syncthreads();
    const double u = uniform53(philox_block(a.seed, a.sample, (uint32_t)t));
    if (wave == 0) {
      bool flag, bad;
      auto val = [&](int x) { return (double)wq[x]; };
      const int site = draw_site(val, bsl, nblk, u, a.delta, a.coef, &flag, &bad, lane);
      if (lane == 0) {
        if (bad) atomicOr(&a.ctl[1], (int)DEV_NUMERICAL);
        sel_x = site;
        need_repair = (flag && !bad) ? 1 : 0;
        if (flag) atomicAdd(&a.counters[0], 1ull);
      }
    }
    __syncthreads();

    if (need_repair) {  // float64 redraw, same uniform
      all_weights<C, true>(a, t, gm, gcf, gc64, occ, a.wr, bsl, tid);
      __syncthreads();
      if (wave == 0) {
        bool flag, bad;
        auto val = [&](int x) { return a.wr[x]; };
        const int site = draw_site(val, bsl, nblk, u, 0.0, 0.0, &flag, &bad, lane);
        if (lane == 0) {
          if (bad) {
            atomicOr(&a.ctl[1], (int)DEV_NUMERICAL);
          } else {
            if (site != sel_x) atomicAdd(&a.counters[1], 1ull);
            sel_x = site;
          }
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
  const int nblk = L_pad / 32;
  size_t b = (wg_lds_bytes<C>(N) + 15) / 16 * 16;
  b += (size_t)nblk * 4;
  b = (b + 7) / 8 * 8;
  b += (size_t)nblk * 8;
  return b;
}

}  // namespace

size_t plain_scratch_bytes(const Dims& d) {
  const size_t es = d.cplx ? 16 : 8;
  size_t b = 4 * (size_t)d.N * d.N * es;  // Li, P, each in two layouts
  b += (size_t)d.N * 4;                   // xs
  b += (size_t)d.L_pad * 8;           // wq
  b += (size_t)d.L_pad * 8;           // wr
  b += 64;                            // ld
  return (b + 255) / 256 * 256 + 1024;
}

void launch_plain(const Dims& d, const void* u64, const void* u64t,
                  const void* ubulk_t, uint64_t seed, uint64_t sample,
                  int n_keep, double delta, double coef, void* scratch, int32_t* x_out,
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
  a.F = take(4 * (size_t)d.N * d.N * es);
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
  a.coef = d.bulk64 ? 0.0 : coef;
  a.seed = seed;
  a.sample = sample;
  auto go = [&](auto kern, size_t lds) {
    allow_lds(kern, lds);
    hipLaunchKernelGGL(kern, dim3(1), dim3(PT), lds, st, a);
  };
  if (d.cplx) {
    const size_t lds = plain_lds<true>(d.N, d.L_pad);
    if (d.bulk64)
      go(plain_kernel<true, true>, lds);
    else
      go(plain_kernel<true, false>, lds);
  } else {
    const size_t lds = plain_lds<false>(d.N, d.L_pad);
    if (d.bulk64)
      go(plain_kernel<false, true>, lds);
    else
      go(plain_kernel<false, false>, lds);
  }
}

}  // namespace ffsk
