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
// A draw is flagged when u*T is within the guard threshold of either end of
// the chosen site's interval: max(delta*T, coef*sqrt(sum_b B_b^2)), B_b the
// float64 block sums.  The second term follows the float32 CDF error: each
// weight carries a relative error of order 2^-24 sqrt(K) with independent
// signs from site to site, so the running sums err by about
// 2^-24 sqrt(K) sqrt(sum_x w(x)^2) <= 2^-24 sqrt(K) sqrt(sum_b B_b^2) (a
// block's squared weights sum to at most its squared sum); coef carries
// that scale times a safety factor fixed per bulk mode.  The flagging
// wavefront queues the draw and lays out its
// dense float64 Gamma; the float64 weights of all flagged draws of the step
// are then formed together (repair_mma_*) and each flagged draw is redone
// with the same u by the next factor launch, before it absorbs the draw.
#include "cx.h"
#include "factor_blk.h"
#include "args.h"
#include "ffs_internal.h"

namespace ffsk {

namespace {


constexpr int DRAW_WAVES = 4;  // samples (wavefronts) per workgroup

// Draw of sample s by one wavefront (lane); shp[64] is this wavefront's LDS
// scratch.
__device__ inline void draw_one(const DArgs& a, int s, int lane, double* shp) {
  const int nblk = a.L_pad / 32;
  int32_t* xrow = a.xs + (size_t)s * a.N;
  uint32_t* oc = a.occ + (size_t)s * nblk;
  if (lane == 0) a.fslot[s] = -1;  // set below when the draw is flagged
  if (a.t < a.n_forced) {  // teacher forcing (test hook)
    if (lane == 0) {
      const int x = a.forced[a.t];
      xrow[a.t] = x;
      atomicOr(&oc[x >> 5], 1u << (x & 31));
    }
    return;
  }
  // the sample's uniform does not depend on the weights: formed while the
  // block sums load
  const Words wd = philox_block(a.seed, sample_index(a.sid, a.first, s), (uint32_t)a.t);
  const double* bs = a.bsum + (size_t)s * nblk;
  // Lane l owns blocks [l*q, min((l+1)*q, nblk)), q = ceil(nblk/64); trailing
  // lanes may own none.  Up to kCached of them stay in registers for the
  // owner's search below.
  constexpr int kCached = 4;
  const int q = (nblk + 63) / 64;
  const int b0 = lane * q;
  const int bn = max(0, min(q, nblk - b0));
  double bc[kCached];
#pragma unroll
  for (int j = 0; j < kCached; ++j) bc[j] = (j < bn) ? bs[b0 + j] : 0.0;
  double P = 0.0, P2 = 0.0;
#pragma unroll
  for (int j = 0; j < kCached; ++j)
    if (j < bn) {
      P += bc[j];
      P2 += bc[j] * bc[j];
    }
  for (int j = kCached; j < bn; ++j) {
    const double v = bs[b0 + j];
    P += v;
    P2 += v * v;
  }
  shp[lane] = P;
  wave_sync();
  // Chunk bounds: every lane forms the running sums of the chunk totals in
  // ascending chunk order (the same additions a single sequential pass
  // makes), lo_l before its own chunk and T over all of them.
  double lo_l = 0.0, T = 0.0;
#pragma unroll 16
  for (int l = 0; l < 64; ++l) {
    const double v = shp[l];
    if (l < lane) lo_l += v;
    T += v;
  }
  const double hi_l = lo_l + P;
  if (!(T > 0.0) || !isfinite(T)) {
    if (lane == 0) {
      atomicOr(&a.ctl[1], (int)DEV_NUMERICAL);
      xrow[a.t] = 0;
    }
    return;
  }
  const double target = uniform53(wd) * T;
  // guard threshold (any lane's reduction order will do: it is compared,
  // never accumulated into a result)
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) P2 += __shfl_xor(P2, o, 64);
  const double thr = fmax(a.delta * T, a.coef * sqrt(P2));
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
  int site = 0;
  if (lane == owner) {
  // ---- block inside the owner's chunk ----
  const double base_lo = lo_l, base_hi = hi_l;
  double Cprev = base_lo, Cb = base_hi, Q = 0.0;
  int blk = -1, lastb = -1;
  for (int j = 0; j < bn; ++j) {
    double v = 0.0;
#pragma unroll
    for (int c = 0; c < kCached; ++c)
      if (c == j) v = bc[c];
    if (j >= kCached) v = bs[b0 + j];
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
  if (fmin(target - lo, hi - target) < thr) flag = true;
  site = gb * 32 + x;
  }  // owner lane
  site = __shfl(site, owner, 64);
  const bool fl = __shfl((int)flag, owner, 64) != 0;
  if (!fl) {
    if (lane == 0) {
      xrow[a.t] = site;
      atomicOr(&oc[site >> 5], 1u << (site & 31));
    }
    return;
  }
  // flagged: queue it and lay out its dense float64 Gamma for the redraw
  int slot = 0;
  if (lane == 0) {
    xrow[a.t] = site;
    slot = atomicAdd(&a.ctl[0], 1);
    a.flag_list[slot] = s;
    a.fslot[s] = slot;
    atomicAdd(&a.counters[0], 1ull);
  }
  slot = __shfl(slot, 0, 64);
  const int32_t* pm = a.perm + (size_t)s * a.N;
  const int32_t* cm = a.cmap ? a.cmap + (size_t)s * a.N : nullptr;
  if (a.cplx) {
    double2* g = reinterpret_cast<double2*>(a.g64) + (size_t)slot * a.Np;
    const double2* bv = reinterpret_cast<const double2*>(a.beta) + (size_t)s * a.N;
    for (int k = lane; k < a.Np; k += 64) g[k] = make_double2(0.0, 0.0);
    __threadfence_block();  // the zeros land before any lane's scatter
    wave_sync();
    for (int i = lane; i <= a.t; i += 64)
      g[cm ? cm[pm[i]] : pm[i]] = (i == a.t) ? make_double2(1.0, 0.0) : make_double2(-bv[i].x, -bv[i].y);
  } else {
    double* g = reinterpret_cast<double*>(a.g64) + (size_t)slot * a.Np;
    const double* bv = reinterpret_cast<const double*>(a.beta) + (size_t)s * a.N;
    for (int k = lane; k < a.Np; k += 64) g[k] = 0.0;
    __threadfence_block();  // the zeros land before any lane's scatter
    wave_sync();
    for (int i = lane; i <= a.t; i += 64) g[cm ? cm[pm[i]] : pm[i]] = (i == a.t) ? 1.0 : -bv[i];
  }
}

// ------------------------------------------------------------- repair ----

__global__ __launch_bounds__(64 * DRAW_WAVES) void draw_kernel(DArgs a) {
  __shared__ double sh_p[DRAW_WAVES][64];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int s = blockIdx.x * DRAW_WAVES + wv;
  if (s >= a.S) return;  // whole wavefront exits together
  draw_one(a, s, lane, sh_p[wv]);
}

// Grouped draw: one wavefront per (instance, sample) item.
__global__ __launch_bounds__(64 * DRAW_WAVES) void draw_group_kernel(const GInst* inst, GList l) {
  __shared__ double sh_p[DRAW_WAVES][64];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int item = blockIdx.x * DRAW_WAVES + wv; item < l.total;
       item += gridDim.x * DRAW_WAVES) {
    const int k = glist_find(l, item);
    const GInst* I = inst + l.ids[k];
    const int t = I->t;
    if (t < 0 || t >= I->n_keep) continue;
    DArgs a = I->da;
    a.t = t;
    draw_one(a, item - l.pre[k], lane, sh_p[wv]);
  }
}

// Float64 weights of all flagged draws of the step as one product on the
// FP64 matrix cores: V[x, f] = sum_k U[x, k] G[f][k] over the dense K = Np,
// so U is streamed once per 32 flagged draws however many there are (the
// unused columns carry zeros).  One wavefront per 64-site chunk (RCHUNK) and
// 32 flagged draws: four 16-row tiles, two 16-column tiles, so a step with a
// single flagged draw spreads the U stream over L_pad / 64 workgroups.
// v_mfma_f64_16x16x4f64 operands: A[l%16][l/16], B[l/16][l%16], D register r
// of lane l = D[l/16 + 4r][l%16].  Each group of 16 k takes k = k0 + 4*(l/16)
// + j for MFMA j = 0..3 in both operands (the same k for A and B, so the sum
// is over all 16), which lets a lane read 4 consecutive Gamma entries.  w =
// |v|^2, occupied sites 0; the chunk sum in a fixed order (lane, then the 4
// lanes of a column).
template <bool C>
__device__ inline void repair_mma_tile(const RArgs& a, int bx, int by, int gy) {
  using X = Cx<C>;
  using T = typename X::T;
  using M = Mma<C>;
  const int count = a.ctl[0];
  const int lane = threadIdx.x & 63;
  const int li = lane & 15, lg = lane >> 4;
  const int nblk = a.L_pad / 32;
  const int nch = a.L_pad / RCHUNK;
  const T* U = reinterpret_cast<const T*>(a.u64t);  // [N][L_pad]
  const T* G = reinterpret_cast<const T*>(a.g64);   // [slot][Np]
  const int x0 = bx * RCHUNK;
  for (int f0 = by * 32; f0 < count; f0 += gy * 32) {
    typename M::Acc acc[4][2];
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) {
      M::zero(acc[rt][0]);
      M::zero(acc[rt][1]);
    }
    const int fa = f0 + li, fb = f0 + 16 + li;
    const bool va = fa < count, vb = fb < count;
    const T* ga = G + (size_t)(va ? fa : 0) * a.Np;
    const T* gb = G + (size_t)(vb ? fb : 0) * a.Np;
    // Real operands: two 16-wide k groups per round trip (loads of both
    // issued first), the products in the same k order as one group at a
    // time, and two register buffers -- the loads of the next round trip
    // are issued before the products of the current one, so their latency
    // overlaps the MFMAs.  The second 16-column tile is skipped when it
    // holds no flagged draw (its columns are never stored).
    constexpr int HG = C ? 1 : 2;
    constexpr int KS = 16 * HG;
    const bool two_ct = f0 + 16 < count;
    struct Ops {
      T av[HG][4][4], bv[HG][2][4];
    };
    auto load = [&](Ops& o, int k0) {
#pragma unroll
      for (int h = 0; h < HG; ++h) {
        const bool hv = h == 0 || k0 + 16 < a.K;
        const int kb = k0 + 16 * h + 4 * lg;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int k = kb + j;
          const bool kv = k < a.K && hv;
          const T* col = U + (size_t)(kv ? k : 0) * a.L_pad + x0 + li;
#pragma unroll
          for (int rt = 0; rt < 4; ++rt) o.av[h][rt][j] = kv ? col[16 * rt] : X::zero();
          o.bv[h][0][j] = (kv && va) ? ga[k] : X::zero();
          o.bv[h][1][j] = (kv && vb) ? gb[k] : X::zero();
        }
      }
    };
    auto mma = [&](const Ops& o, int k0) {
#pragma unroll
      for (int h = 0; h < HG; ++h) {
        if (h == 1 && !(k0 + 16 < a.K)) break;
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int rt = 0; rt < 4; ++rt) {
            M::mma(acc[rt][0], o.av[h][rt][j], o.bv[h][0][j]);
            if (two_ct) M::mma(acc[rt][1], o.av[h][rt][j], o.bv[h][1][j]);
          }
      }
    };
    if constexpr (!C) {
      Ops o0, o1;
      load(o0, 0);
      for (int k0 = 0; k0 < a.K; k0 += 2 * KS) {
        if (k0 + KS < a.K) load(o1, k0 + KS);
        mma(o0, k0);
        if (k0 + KS >= a.K) break;
        if (k0 + 2 * KS < a.K) load(o0, k0 + 2 * KS);
        mma(o1, k0 + KS);
      }
    } else {  // complex operands take twice the registers: one buffer
      for (int k0 = 0; k0 < a.K; k0 += KS) {
        Ops o;
        load(o, k0);
        mma(o, k0);
      }
    }
    // epilogue: lane holds sites x0 + 16 rt + lg + 4 r of columns li, 16 + li
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
      const int f = f0 + 16 * ct + li;
      const bool fv = f < count;
      const int s = fv ? a.flag_list[f] : 0;
      double sum = 0.0;
#pragma unroll
      for (int rt = 0; rt < 4; ++rt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int x = x0 + 16 * rt + lg + 4 * r;
          const bool occd = (a.occ[(size_t)s * nblk + (x >> 5)] >> (x & 31)) & 1u;
          const double w = occd ? 0.0 : X::abs2(M::get(acc[rt][ct], r));
          if (fv) a.wr[(size_t)f * a.L_pad + x] = w;
          sum += w;
        }
      sum += __shfl_xor(sum, 16, 64);
      sum += __shfl_xor(sum, 32, 64);
      if (lg == 0 && fv) a.cs[(size_t)f * nch + bx] = sum;
    }
  }
}

template <bool C>
__global__ __launch_bounds__(64) void repair_mma_kernel(RArgs a) {
  repair_mma_tile<C>(a, blockIdx.x, blockIdx.y, gridDim.y);
}

// Column tiles of 32 flagged draws per 64-site chunk for S samples: the
// grouped launches take at most 2 per chunk (every instance's items share
// one list); a single launch takes enough to give about 1024 workgroups, so
// steps with many flagged draws fill the chip.  Empty tiles exit at once,
// and a tile's results do not depend on how many there are.
__host__ __device__ inline int repair_ctiles(int S) {
  const int c = (S + 31) / 32;
  return c < 2 ? c : 2;
}
inline int repair_ctiles_wide(int S, int nch) {
  const int c = (S + 31) / 32;
  int want = (1024 + nch - 1) / nch;
  if (want < 2) want = 2;
  return c < want ? c : want;
}

template <bool C>
__global__ __launch_bounds__(64) void repair_mma_group_kernel(const GInst* inst, GList l) {
  for (int item = blockIdx.x; item < l.total; item += gridDim.x) {
    const int k = glist_find(l, item);
    const GInst* I = inst + l.ids[k];
    const int t = I->t;
    if (t < 0 || t >= I->n_keep) continue;
    RArgs a = I->ra;
    a.t = t;
    const int local = item - l.pre[k];
    const int gy = repair_ctiles(I->S);
    repair_mma_tile<C>(a, local / gy, local % gy, gy);
  }
}

}  // namespace

DArgs make_dargs(const Dims& d, const Work& w, int S, uint64_t seed,
                 uint64_t first, double delta, double coef, int n_forced) {
  DArgs a;
  a.bsum = w.bsum;
  a.wh = static_cast<const float*>(w.wh);
  a.xs = w.xs;
  a.occ = w.occ;
  a.ctl = w.ctl;
  a.flag_list = w.flag_list;
  a.counters = w.counters;
  a.forced = w.forced;
  a.perm = w.perm;
  a.beta = w.beta;
  a.g64 = w.g64;
  a.cmap = w.cmap;
  a.sid = w.sid;
  a.fslot = w.fslot;
  a.S = S;
  a.L_pad = d.L_pad;
  a.N = d.N;
  a.Np = d.Np;
  a.t = 0;
  a.n_forced = n_forced;
  a.cplx = d.cplx;
  a.delta = delta;
  a.coef = coef;
  a.seed = seed;
  a.first = first;
  return a;
}

RArgs make_rargs(const Dims& d, const Work& w, const void* u64t, uint64_t seed,
                 uint64_t first) {
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
  a.g64 = w.g64;
  a.sid = w.sid;
  a.L_pad = d.L_pad;
  a.N = d.N;
  a.Np = d.Np;
  a.K = d.ldu;
  a.t = 0;
  a.seed = seed;
  a.first = first;
  return a;
}

void launch_draw(const Dims& d, const Work& w, int S, int t, uint64_t seed,
                 uint64_t first, double delta, double coef, int n_forced,
                 hipStream_t st) {
  DArgs a = make_dargs(d, w, S, seed, first, delta, coef, n_forced);
  a.t = t;
  hipLaunchKernelGGL(draw_kernel, dim3((S + DRAW_WAVES - 1) / DRAW_WAVES),
                     dim3(64 * DRAW_WAVES), 0, st, a);
}

void launch_repair(const Dims& d, const Work& w, const void* u64t, int S,
                   int t, uint64_t seed, uint64_t first, hipStream_t st) {
  RArgs a = make_rargs(d, w, u64t, seed, first);
  a.t = t;
  dim3 g1(d.L_pad / RCHUNK, repair_ctiles_wide(S, d.L_pad / RCHUNK));
  if (d.cplx)
    hipLaunchKernelGGL(repair_mma_kernel<true>, g1, dim3(64), 0, st, a);
  else
    hipLaunchKernelGGL(repair_mma_kernel<false>, g1, dim3(64), 0, st, a);
}

int repair_group_items(const Dims& d, int S) { return (d.L_pad / RCHUNK) * repair_ctiles(S); }

void launch_draw_group(const GInst* inst, const GList& l, hipStream_t st) {
  if (l.total == 0) return;
  const int blocks = (l.total + DRAW_WAVES - 1) / DRAW_WAVES;
  hipLaunchKernelGGL(draw_group_kernel, dim3(blocks < 4096 ? blocks : 4096),
                     dim3(64 * DRAW_WAVES), 0, st, inst, l);
}

void launch_repair_group(const GInst* inst, const GList& mma_l, bool cplx, hipStream_t st) {
  if (mma_l.total > 0) {
    const int grid = mma_l.total < 4096 ? mma_l.total : 4096;
    if (cplx)
      hipLaunchKernelGGL(repair_mma_group_kernel<true>, dim3(grid), dim3(64), 0, st, inst, mma_l);
    else
      hipLaunchKernelGGL(repair_mma_group_kernel<false>, dim3(grid), dim3(64), 0, st, inst, mma_l);
  }
}

}  // namespace ffsk
