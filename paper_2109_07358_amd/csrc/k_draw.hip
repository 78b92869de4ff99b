// Batched path: inverse-CDF draw with its near-tie guard, and the float64
// redraw of the draws the guard flagged.
//
// Draw rule (same as the oracle's): x = the first site, in ascending order,
// whose running float64 sum F exceeds u*T, T the float64 total and u the
// 53-bit uniform of the (sample, step) Philox block.  Running sums are built
// in three fixed-order levels so that every level agrees exactly with the
// next at its boundaries:
//   lane chunks  -- lane l of the sample's wavefront owns q = nblk/64
//                   consecutive 32-site blocks; base_{l+1} = base_l + P_l,
//                   summed sequentially over lanes;
//   blocks       -- inside the selected chunk, C_j = base_l + (sequential
//                   in-chunk prefix), the chunk's last block taking base_{l+1};
//   sites        -- inside the selected block, F = C_{j-1} + (sequential
//                   prefix of the float32 weights), the last site taking C_j.
// A draw is flagged when u*T is within delta*T of either end of the chosen
// site's interval; flagged draws are redone by repair_* from float64
// weights with the same u.
#include "cx.h"
#include "ffs_internal.h"

namespace ffsk {

namespace {

struct DArgs {
  const double* bsum;  // [S_pad][nblk]
  const float* wh;     // [S_pad][L_pad]
  int32_t* xs;         // [S_pad][N]
  uint32_t* occ;       // [S_pad][nblk]
  int32_t* ctl;        // [0] flag count, [1] status
  int32_t* flag_list;
  unsigned long long* counters;
  const int32_t* forced;
  int S, L_pad, N, t, n_forced;
  double delta;
  uint64_t seed, first;
};

constexpr int DRAW_WAVES = 4;  // samples (wavefronts) per workgroup

__global__ __launch_bounds__(64 * DRAW_WAVES) void draw_kernel(DArgs a) {
  __shared__ double sh_p[DRAW_WAVES][64];
  __shared__ double sh_base[DRAW_WAVES][65];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int s = blockIdx.x * DRAW_WAVES + wv;
  if (s >= a.S) return;  // whole wavefront exits together
  const int nblk = a.L_pad / 32;
  int32_t* xrow = a.xs + (size_t)s * a.N;
  uint32_t* oc = a.occ + (size_t)s * nblk;
  if (a.t < a.n_forced) {  // teacher forcing (test hook)
    if (lane == 0) {
      const int x = a.forced[a.t];
      xrow[a.t] = x;
      atomicOr(&oc[x >> 5], 1u << (x & 31));
    }
    return;
  }
  const double* bs = a.bsum + (size_t)s * nblk;
  // Lane l owns blocks [l*q, min((l+1)*q, nblk)), q = ceil(nblk/64); trailing
  // lanes may own none.
  const int q = (nblk + 63) / 64;
  const int b0 = lane * q;
  const int bn = max(0, min(q, nblk - b0));
  double P = 0.0;
  for (int j = 0; j < bn; ++j) P += bs[b0 + j];
  sh_p[wv][lane] = P;
  wave_sync();
  if (lane == 0) {
    double base = 0.0;
    for (int l = 0; l < 64; ++l) {
      sh_base[wv][l] = base;
      base += sh_p[wv][l];
    }
    sh_base[wv][64] = base;
  }
  wave_sync();
  const double T = sh_base[wv][64];
  if (!(T > 0.0) || !isfinite(T)) {
    if (lane == 0) {
      atomicOr(&a.ctl[1], (int)DEV_NUMERICAL);
      xrow[a.t] = 0;
    }
    return;
  }
  const Words wd = philox_block(a.seed, a.first + (uint64_t)s, (uint32_t)a.t);
  const double target = uniform53(wd) * T;
  const double lo_l = sh_base[wv][lane], hi_l = sh_base[wv][lane + 1];
  const unsigned long long hit = __ballot(lo_l <= target && target < hi_l && bn > 0);
  bool flag = false;
  int owner;
  if (hit) {
    owner = __builtin_ctzll(hit);
  } else {  // u*T at or above the total (rounding): last chunk with mass
    flag = true;
    const unsigned long long nz = __ballot(P > 0.0 && bn > 0);
    owner = 63 - __builtin_clzll(nz);
  }
  if (lane != owner) return;
  // ---- block inside the owner's chunk ----
  const double base_lo = sh_base[wv][lane], base_hi = sh_base[wv][lane + 1];
  double Cprev = base_lo, Cb = base_hi, Q = 0.0;
  int blk = -1, lastb = -1;
  for (int j = 0; j < bn; ++j) {
    const double v = bs[b0 + j];
    Q += v;
    const double C = (j == bn - 1) ? base_hi : base_lo + Q;
    if (v > 0.0) {
      lastb = j;
      if (blk < 0 && C > target) {
        blk = j;
        Cb = C;
        break;
      }
    }
    Cprev = C;
  }
  if (blk < 0) {  // rounding disagreement at the chunk end
    flag = true;
    blk = lastb;
    Q = 0.0;
    Cprev = base_lo;
    for (int j = 0; j < blk; ++j) {
      Q += bs[b0 + j];
      Cprev = base_lo + Q;
    }
    Cb = (blk == bn - 1) ? base_hi : base_lo + (Q + bs[b0 + blk]);
  }
  const int gb = b0 + blk;
  // ---- site inside the block ----
  const float4* wp = reinterpret_cast<const float4*>(a.wh + (size_t)s * a.L_pad + (size_t)gb * 32);
  float w[32];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const float4 v = wp[k];
    w[4 * k] = v.x;
    w[4 * k + 1] = v.y;
    w[4 * k + 2] = v.z;
    w[4 * k + 3] = v.w;
  }
  double R = 0.0, prev = Cprev, lo = Cprev, hi = Cb;
  int x = -1, last = -1;
#pragma unroll
  for (int j = 0; j < 32; ++j) {
    const double wj = (double)w[j];
    R += wj;
    const double F = (j == 31) ? Cb : Cprev + R;
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
  if (x < 0) {  // rounding disagreement at the block end
    flag = true;
    x = last;
    lo = hi = target;
  }
  if (fmin(target - lo, hi - target) < a.delta * T) flag = true;
  const int site = gb * 32 + x;
  xrow[a.t] = site;
  if (flag) {
    const int slot = atomicAdd(&a.ctl[0], 1);
    a.flag_list[slot] = s;
    atomicAdd(&a.counters[0], 1ull);
  } else {
    atomicOr(&oc[site >> 5], 1u << (site & 31));
  }
}

// ------------------------------------------------------------- repair ----
struct RArgs {
  const void* u64t;    // [N][L_pad] column-major float64 / complex128
  const int32_t* perm;
  const void* beta;
  int32_t* xs;
  uint32_t* occ;
  int32_t* ctl;
  const int32_t* flag_list;
  unsigned long long* counters;
  double* wr;          // [S_pad][L_pad] float64 weights of flagged draws
  double* cs;          // [S_pad][nch]   their 256-site chunk sums
  int L_pad, N, t;
  uint64_t seed, first;
};

// Float64 weights of the flagged draws: grid (L_pad/256 chunks, slots);
// v(y) = sum_{i<=t} U[y, m_i] g_i, g_t = 1, g_i = -beta_i; w = |v|^2 with
// occupied sites zeroed; chunk sums by a fixed-order tree.
template <bool C>
__global__ __launch_bounds__(256) void repair_weights_kernel(RArgs a) {
  using X = Cx<C>;
  using T = typename X::T;
  __shared__ T gc[1024];
  __shared__ int gm[1024];
  __shared__ double red[256];
  const int tid = threadIdx.x;
  const int count = a.ctl[0];
  const int nblk = a.L_pad / 32;
  const int nch = a.L_pad / RCHUNK;
  const T* U = reinterpret_cast<const T*>(a.u64t);
  const int x = blockIdx.x * RCHUNK + tid;
  for (int f = blockIdx.y; f < count; f += gridDim.y) {
    const int s = a.flag_list[f];
    const int32_t* pm = a.perm + (size_t)s * a.N;
    const T* bv = reinterpret_cast<const T*>(a.beta) + (size_t)s * a.N;
    for (int i = tid; i <= a.t; i += 256) {
      gm[i] = pm[i];
      gc[i] = (i == a.t) ? X::one() : X::neg(bv[i]);
    }
    __syncthreads();
    T acc = X::zero();
    int i = 0;
    for (; i + 8 <= a.t + 1; i += 8) {
      T u[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) u[k] = U[(size_t)gm[i + k] * a.L_pad + x];
#pragma unroll
      for (int k = 0; k < 8; ++k) acc = X::fma(u[k], gc[i + k], acc);
    }
    for (; i <= a.t; ++i) acc = X::fma(U[(size_t)gm[i] * a.L_pad + x], gc[i], acc);
    const bool occd = (a.occ[(size_t)s * nblk + (x >> 5)] >> (x & 31)) & 1u;
    const double w = occd ? 0.0 : X::abs2(acc);
    a.wr[(size_t)f * a.L_pad + x] = w;
    red[tid] = w;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
      if (tid < h) red[tid] += red[tid + h];
      __syncthreads();
    }
    if (tid == 0) a.cs[(size_t)f * nch + blockIdx.x] = red[0];
    __syncthreads();
  }
}

// Redraw with the same u from the float64 weights: chunk sums scanned in
// order, then the chunk's sites in order (last site takes the chunk end).
__global__ __launch_bounds__(256) void repair_draw_kernel(RArgs a) {
  __shared__ double csl[65536 / RCHUNK];
  __shared__ double wl[RCHUNK];
  __shared__ int sel_chunk;
  __shared__ double sel_lo, sel_hi;
  const int tid = threadIdx.x;
  const int count = a.ctl[0];
  const int nblk = a.L_pad / 32;
  const int nch = a.L_pad / RCHUNK;
  for (int f = blockIdx.x; f < count; f += gridDim.x) {
    const int s = a.flag_list[f];
    for (int c = tid; c < nch; c += 256) csl[c] = a.cs[(size_t)f * nch + c];
    __syncthreads();
    double target = 0.0;
    if (tid == 0) {
      double T64 = 0.0;
      for (int c = 0; c < nch; ++c) T64 += csl[c];
      target = uniform53(philox_block(a.seed, a.first + (uint64_t)s, (uint32_t)a.t)) * T64;
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
      sel_chunk = ch;
      sel_lo = Cc;
      sel_hi = Cn;
    }
    __syncthreads();
    const int ch = sel_chunk;
    if (ch >= 0) wl[tid] = a.wr[(size_t)f * a.L_pad + (size_t)ch * RCHUNK + tid];
    __syncthreads();
    if (tid == 0) {
      int32_t* xrow = a.xs + (size_t)s * a.N;
      int site;
      if (ch < 0) {  // no float64 mass: report, keep the first draw
        atomicOr(&a.ctl[1], (int)DEV_NUMERICAL);
        site = xrow[a.t];
      } else {
        const double Cc = sel_lo, Cn = sel_hi;
        double Pp = 0.0;
        int xx = -1, last = -1;
        for (int j = 0; j < RCHUNK; ++j) {
          const double wj = wl[j];
          Pp += wj;
          const double F = (j == RCHUNK - 1) ? Cn : Cc + Pp;
          if (wj > 0.0) {
            last = j;
            if (xx < 0 && F > target) xx = j;
          }
        }
        if (xx < 0) xx = last;
        site = ch * RCHUNK + xx;
      }
      if (xrow[a.t] != site) atomicAdd(&a.counters[1], 1ull);
      xrow[a.t] = site;
      atomicOr(&a.occ[(size_t)s * nblk + (site >> 5)], 1u << (site & 31));
    }
    __syncthreads();
  }
}

}  // namespace

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
  a.L_pad = d.L_pad;
  a.N = d.N;
  a.t = t;
  a.n_forced = n_forced;
  a.delta = delta;
  a.seed = seed;
  a.first = first;
  hipLaunchKernelGGL(draw_kernel, dim3((S + DRAW_WAVES - 1) / DRAW_WAVES),
                     dim3(64 * DRAW_WAVES), 0, st, a);
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
  a.cs = w.cs;
  a.L_pad = d.L_pad;
  a.N = d.N;
  a.t = t;
  a.seed = seed;
  a.first = first;
  const int slots = S < FMAX ? S : FMAX;
  dim3 g1(d.L_pad / RCHUNK, slots);
  if (d.cplx)
    hipLaunchKernelGGL(repair_weights_kernel<true>, g1, dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL(repair_weights_kernel<false>, g1, dim3(256), 0, st, a);
  hipLaunchKernelGGL(repair_draw_kernel, dim3(slots), dim3(256), 0, st, a);
}

}  // namespace ffsk
