// Metropolis conditional update (SI S-7): for large L the all-site weights
// of a step are replaced by a short Markov chain on the single variable x_t.
// The chain targets the same conditional, w(y) = |v_t(y)|^2 with
// v_t(y) = U[y, m_t] - sum_{i<t} beta_i U[y, m_i] (Eq. (3), h = (-beta, 1)),
// and accepts a proposal y over the current site c with probability
// min(1, w(y) / w(c)); occupied sites weigh 0.  Per step the work is
// m_cond evaluations of one t-term sum, so a sample costs O(m_cond N^2 +
// N^3) instead of O(L N^2).
//
// The chain starts at the anchor of column m_t -- the first row of largest
// |U[., m_t]|^2, where the new orbital's weight concentrates -- with its
// weight (0 if occupied).  Iteration j of step t of sample s uses the Philox
// block (seed, s, t, 2 + j) (word 3 >= 2: disjoint from the sampler's stream
// 0 and the DPP selection's stream 1).  Its words 0,1 pick the proposal by
// 64-bit multiply-high -- uniform over the L sites when radius == 0, else
// c + d with d uniform in [-radius, -1] u [1, radius], wrapped modulo L
// (both symmetric) -- and words 2,3 give u (53 bits); y is accepted when
// u w(c) < w(y).  A chain that ends on a site of weight 0 moves to the
// nearest free site of positive weight (distance 1, 2, ... from it, the
// lower side first), and reports NUMERICAL if there is none.
//
// One wavefront per sample, all in float64.  With global proposals (radius
// 0) the proposals do not depend on the chain's site, so the weights of 8
// proposals are formed together (their row loads in flight at once), each
// in the same order as one at a time, and then accepted or rejected in turn.
#include "cx.h"
#include "ffs_internal.h"

namespace ffsk {
namespace {

// The t-term sum of one proposal: term i = lane + 64 r sits in register
// slot r of its lane (loaded once per step), so a proposal costs one round
// of independent row loads.  Lanes sum their slots in ascending i, then a
// fixed butterfly combines the lanes.
constexpr int kSlots = 16;  // 64 * 16 = 1024 terms, the largest N

template <bool C>
struct StepTerms {
  typename Cx<C>::T b[kSlots];
  int c[kSlots];
  int ct;  // column m_t
};

template <bool C>
__device__ inline double mh_weight(const typename Cx<C>::T* U, int N, const StepTerms<C>& st,
                                   int t, int y, int lane) {
  using X = Cx<C>;
  using T = typename X::T;
  const T* row = U + (size_t)y * N;
  T acc = X::zero();
#pragma unroll
  for (int r = 0; r < kSlots; ++r)
    if (lane + 64 * r < t) acc = X::fma(st.b[r], row[st.c[r]], acc);
  acc = wave_sum<C>(acc);
  return X::abs2(X::sub(row[st.ct], acc));
}

__device__ inline bool occupied(const uint32_t* occ, int y) {
  return (occ[y >> 5] >> (y & 31)) & 1u;
}

// GLOBAL: radius == 0 (the batched proposal loop below), else local moves.
template <bool C, bool GLOBAL>
__global__ __launch_bounds__(256) void mh_kernel(const void* u64, const int32_t* anchor,
                                                 const int32_t* perm_all, const void* beta_all,
                                                 int32_t* xs, int32_t* fslot, uint32_t* occ_all,
                                                 int32_t* ctl,
                                                 unsigned long long* counters, int S, int L,
                                                 int L_pad, int N, int t, int m_cond, int radius,
                                                 uint64_t seed, uint64_t first) {
  using X = Cx<C>;
  using T = typename X::T;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int s = blockIdx.x * 4 + wv;
  if (s >= S) return;  // whole wavefront exits together
  const T* U = reinterpret_cast<const T*>(u64);
  const int32_t* perm = perm_all + (size_t)s * N;
  const T* beta = reinterpret_cast<const T*>(beta_all) + (size_t)s * N;
  uint32_t* occ = occ_all + (size_t)s * (L_pad / 32);
  const uint64_t sample = first + (uint64_t)s;
  StepTerms<C> tm;
#pragma unroll
  for (int r = 0; r < kSlots; ++r) {
    const int i = lane + 64 * r;
    tm.b[r] = i < t ? beta[i] : X::zero();
    tm.c[r] = i < t ? perm[i] : 0;
  }
  tm.ct = perm[t];
  int cur = anchor[tm.ct];
  double wc = occupied(occ, cur) ? 0.0 : mh_weight<C>(U, N, tm, t, cur, lane);
  unsigned long long acc_n = 0;
  // Weights of kBatch sites (0 where !use[b]), each formed in the same
  // order as mh_weight forms it, with every row load of a slot issued before
  // any is used (rows of any site are valid addresses).
  constexpr int kBatch = 8;
  auto batch_weights = [&](const int(&ys)[kBatch], const bool(&use)[kBatch],
                           double(&wy)[kBatch]) {
    const T* rows[kBatch];
    T acc[kBatch];
#pragma unroll
    for (int b = 0; b < kBatch; ++b) {
      rows[b] = U + (size_t)ys[b] * N;
      acc[b] = X::zero();
    }
#pragma unroll
    for (int r = 0; r < kSlots; ++r)
      if (lane + 64 * r < t) {
        T vals[kBatch];
#pragma unroll
        for (int b = 0; b < kBatch; ++b) vals[b] = rows[b][tm.c[r]];
#pragma unroll
        for (int b = 0; b < kBatch; ++b) acc[b] = X::fma(tm.b[r], vals[b], acc[b]);
      }
#pragma unroll
    for (int b = 0; b < kBatch; ++b) {
      wy[b] = 0.0;
      if (use[b]) wy[b] = X::abs2(X::sub(rows[b][tm.ct], wave_sum<C>(acc[b])));
    }
  };
  auto accept = [&](int y, double wy, double u) {
    if (!(u * wc < wy)) return 0;
    cur = y;
    wc = wy;
    ++acc_n;
    return 1;
  };
  if constexpr (GLOBAL) {
    // Proposals do not depend on the chain's site: kBatch of them at once,
    // then accepted or rejected in order.
    for (int j0 = 0; j0 < m_cond; j0 += kBatch) {
      int ys[kBatch];
      double us[kBatch], wy[kBatch];
      bool use[kBatch];
#pragma unroll
      for (int b = 0; b < kBatch; ++b) {
        const int j = j0 + b;
        const Words w = philox_stream(seed, sample, (uint32_t)t, 2u + (uint32_t)(j < m_cond ? j : 0));
        const uint64_t v = ((uint64_t)w.w1 << 32) | w.w0;
        ys[b] = (int)(uint64_t)(((unsigned __int128)v * (uint64_t)L) >> 64);
        us[b] = uniform53(w);
        use[b] = j < m_cond && !occupied(occ, ys[b]);
      }
      batch_weights(ys, use, wy);
#pragma unroll
      for (int b = 0; b < kBatch; ++b)
        if (j0 + b < m_cond) accept(ys[b], wy[b], us[b]);
    }
  } else {
    // Local moves depend on the chain's site: one proposal at a time.  (A
    // tree of the 7 sites three iterations can propose, weighed at once,
    // measured slower: 2.3 times the weights and a lower occupancy.)
    for (int j = 0; j < m_cond; ++j) {
      const Words w = philox_stream(seed, sample, (uint32_t)t, 2u + (uint32_t)j);
      const uint64_t v = ((uint64_t)w.w1 << 32) | w.w0;
      const int r = (int)(uint64_t)(((unsigned __int128)v * (uint64_t)(2 * radius)) >> 64);
      const int dlt = r < radius ? r - radius : r - radius + 1;
      int y = (int)(((int64_t)cur + dlt) % L);
      if (y < 0) y += L;
      const double wy = occupied(occ, y) ? 0.0 : mh_weight<C>(U, N, tm, t, y, lane);
      accept(y, wy, uniform53(w));
    }
  }
  if (!(wc > 0.0)) {  // nearest free site of positive weight, lower side first
    const int c0 = cur;
    int found = -1;
    if constexpr (GLOBAL) {
      // the same search kBatch candidates at a time: candidate k is
      // c0 - (k/2 + 1) for even k, c0 + (k/2 + 1) for odd k; the first of
      // positive weight in k order is the one the one-by-one search finds
      for (int k0 = 0; found < 0 && k0 / 2 + 1 < L; k0 += kBatch) {
        int ys[kBatch];
        bool use[kBatch];
        double wy[kBatch];
#pragma unroll
        for (int b = 0; b < kBatch; ++b) {
          const int k = k0 + b, dist = k / 2 + 1;
          const int y = (k & 1) ? c0 + dist : c0 - dist;
          use[b] = dist < L && y >= 0 && y < L && !occupied(occ, y);
          ys[b] = use[b] ? y : c0;
        }
        batch_weights(ys, use, wy);
#pragma unroll
        for (int b = 0; b < kBatch; ++b)
          if (found < 0 && wy[b] > 0.0) found = ys[b];
      }
    } else {
      for (int dist = 1; dist < L && found < 0; ++dist) {
        const int ys[2] = {c0 - dist, c0 + dist};
        for (int k = 0; k < 2 && found < 0; ++k) {
          const int y = ys[k];
          if (y < 0 || y >= L || occupied(occ, y)) continue;
          if (mh_weight<C>(U, N, tm, t, y, lane) > 0.0) found = y;
        }
      }
    }
    if (found < 0) {
      for (int y = 0; y < L && found < 0; ++y)
        if (!occupied(occ, y)) found = y;
      if (lane == 0) atomicOr(&ctl[1], (int)DEV_NUMERICAL);
    }
    cur = found;
  }
  if (lane == 0) {
    fslot[s] = -1;  // no float64 redraw pending for the factor launch
    xs[(size_t)s * N + t] = cur;
    occ[cur >> 5] |= 1u << (cur & 31);
    atomicAdd(&counters[2], acc_n);
  }
}

}  // namespace

void launch_mh(const Dims& d, const Work& w, const void* u64, const int32_t* anchor, int S,
               int t, int m_cond, int radius, uint64_t seed, uint64_t first, hipStream_t st) {
  const dim3 grid((unsigned)((S + 3) / 4));
  auto go = [&](auto kern) {
    hipLaunchKernelGGL(kern, grid, dim3(256), 0, st, u64, anchor, w.perm, w.beta, w.xs, w.fslot,
                       w.occ, w.ctl, w.counters, S, d.L, d.L_pad, d.N, t, m_cond, radius, seed,
                       first);
  };
  if (d.cplx) {
    if (radius == 0)
      go(mh_kernel<true, true>);
    else
      go(mh_kernel<true, false>);
  } else {
    if (radius == 0)
      go(mh_kernel<false, true>);
    else
      go(mh_kernel<false, false>);
  }
}

}  // namespace ffsk
