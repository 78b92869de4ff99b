// Batched path: the separate draw launches (per-step resolution), the
// float64 product V = U Gamma of flagged draws on the FP64 matrix cores, and
// the end-of-call float64 check of the draws a deferred call recorded.  The
// draw itself and the float64 redraw rule are in draw.h.
#include "cx.h"
#include "factor_blk.h"
#include "args.h"
#include "draw.h"
#include "ffs_internal.h"

namespace ffsk {

namespace {

constexpr int DRAW_WAVES = 4;  // samples (wavefronts) per workgroup

__global__ __launch_bounds__(64 * DRAW_WAVES) void draw_kernel(DArgs a) {
  __shared__ double sh_p[DRAW_WAVES][64];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int s = blockIdx.x * DRAW_WAVES + wv;
  if (s >= a.S) return;  // whole wavefront exits together
  draw_one<false>(a, s, lane, sh_p[wv]);
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
    draw_one<false>(a, item - l.pre[k], lane, sh_p[wv]);
  }
}

// ------------------------------------------------------------- repair ----

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
// lanes of a column).  Complex products take Gauss's three-multiplication
// form (RepairMma<true>).

// Matrix-core steps of the float64 redraw product.  Real: one MFMA per k
// group.  Complex: P1 = Ur Gr, P2 = Ui Gi and P3 = (Ur + Ui)(Gr + Gi) in
// three accumulators (three MFMAs where the direct complex product takes
// four), and v = (P1 - P2, (P3 - P1) - P2).
template <bool C>
struct RepairMma : Mma<false> {};
template <>
struct RepairMma<true> {
  struct Acc {
    doublex4 p1, p2, p3;
  };
  __device__ static void zero(Acc& a) {
    a.p1 = doublex4{0.0, 0.0, 0.0, 0.0};
    a.p2 = a.p1;
    a.p3 = a.p1;
  }
  __device__ static void mma(Acc& acc, double2 a, double2 b) {
    acc.p1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.x, acc.p1, 0, 0, 0);
    acc.p2 = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, b.y, acc.p2, 0, 0, 0);
    acc.p3 = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x + a.y, b.x + b.y, acc.p3, 0, 0, 0);
  }
  __device__ static double2 get(const Acc& a, int r) {
    return make_double2(a.p1[r] - a.p2[r], (a.p3[r] - a.p1[r]) - a.p2[r]);
  }
};

template <bool C>
__device__ inline void repair_mma_tile(const RArgs& a, int bx, int by, int gy) {
  using X = Cx<C>;
  using T = typename X::T;
  using M = RepairMma<C>;
  int count = a.ctl[0];
  if (a.occ_rec) count = max(0, min(min(count, a.rec_cap) - a.rec_base, a.rec_span));
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
      const uint32_t* orow = a.occ_rec ? a.occ_rec + (size_t)(fv ? f : 0) * nblk
                                       : a.occ + (size_t)(fv ? a.flag_list[f] : 0) * nblk;
      double sum = 0.0;
#pragma unroll
      for (int rt = 0; rt < 4; ++rt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int x = x0 + 16 * rt + lg + 4 * r;
          const bool occd = (orow[x >> 5] >> (x & 31)) & 1u;
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

// End-of-call check of record rec_base + f (one wavefront): its float64
// site with the draw's u against the float32 site it kept.  A moved site
// counts as changed and lists the sample for a replay; no float64 mass
// reports NUMERICAL (the sample keeps its draw, as per-step resolution does).
__global__ __launch_bounds__(64) void check_records_kernel(VArgs a) {
  __shared__ __align__(16) char lds[(64 + RCHUNK) * 8 + 8 + 3 * 8];
  const int f = blockIdx.x, lane = threadIdx.x;
  const int count = max(0, min(min(a.rec_ctl[0], a.rec_cap) - a.rec_base, a.rec_span));
  if (f >= count) return;
  const int32_t* m = a.rec_meta + 4 * (size_t)(a.rec_base + f);
  const int s = m[0], t = m[1], x32 = m[2];
  const int nch = a.L_pad / RCHUNK;
  const int site = redraw_site(a.cs + (size_t)f * nch, a.wr + (size_t)f * a.L_pad, a.L_pad,
                               a.seed, sample_index(a.sid, a.first, s), t, lane, lds);
  if (lane == 0) {
    if (site < 0) {
      atomicOr(&a.ctl[1], (int)DEV_NUMERICAL);
    } else if (site != x32) {
      atomicAdd(&a.counters[1], 1ull);
      list_replay(a.div, a.rep_ctl, a.rep_row, a.rep_sid, a.row0, a.sid, a.first, s);
    }
  }
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
  a.rec_meta = nullptr;  // per-step resolution (launch_drawfactor sets these)
  a.rec_g = nullptr;
  a.rec_occ = nullptr;
  a.rec_ctl = w.rec_ctl;
  a.div = w.div;
  a.rep_row = w.rep_row;
  a.rep_sid = w.rep_sid;
  a.rec_cap = 0;
  a.row0 = 0;
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
  a.occ_rec = nullptr;
  a.rec_base = 0;
  a.rec_span = 0;
  a.rec_cap = 0;
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

void launch_check_records(const Dims& d, const Work& w, const void* u64t, uint64_t seed,
                          uint64_t first, int row0, hipStream_t st) {
  const size_t es = d.cplx ? 16 : 8;
  const int nblk = d.L_pad / 32;
  for (int base = 0; base < w.rec_cap; base += w.S_pad) {
    const int span = w.rec_cap - base < w.S_pad ? w.rec_cap - base : w.S_pad;
    RArgs a = make_rargs(d, w, u64t, seed, first);
    a.ctl = w.rec_ctl;
    a.g64 = static_cast<char*>(w.rec_g) + (size_t)base * d.Np * es;
    a.occ_rec = w.rec_occ + (size_t)base * nblk;
    a.rec_base = base;
    a.rec_span = span;
    a.rec_cap = w.rec_cap;
    dim3 g1(d.L_pad / RCHUNK, repair_ctiles_wide(span, d.L_pad / RCHUNK));
    if (d.cplx)
      hipLaunchKernelGGL(repair_mma_kernel<true>, g1, dim3(64), 0, st, a);
    else
      hipLaunchKernelGGL(repair_mma_kernel<false>, g1, dim3(64), 0, st, a);
    VArgs v;
    v.rec_meta = w.rec_meta;
    v.rec_ctl = w.rec_ctl;
    v.wr = w.wr;
    v.cs = w.cs;
    v.ctl = w.ctl;
    v.counters = w.counters;
    v.div = w.div;
    v.rep_row = w.rep_row;
    v.rep_sid = w.rep_sid;
    v.rep_ctl = w.rec_ctl;
    v.sid = w.sid;
    v.L_pad = d.L_pad;
    v.rec_base = base;
    v.rec_span = span;
    v.rec_cap = w.rec_cap;
    v.row0 = row0;
    v.seed = seed;
    v.first = first;
    hipLaunchKernelGGL(check_records_kernel, dim3(span), dim3(64), 0, st, v);
  }
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
