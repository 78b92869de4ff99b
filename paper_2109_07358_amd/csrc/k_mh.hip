// Metropolis conditional update (SI S-7): for large L the all-site weights
// of a step are replaced by a short Markov chain on the single variable x_t.
// The chain targets the same conditional, w(y) = |v_t(y)|^2 with
// v_t(y) = U[y, m_t] - sum_{i<t} beta_i U[y, m_i] (Eq. (3), h = (-beta, 1)),
// and accepts a proposal y over the current site c with probability
// min(1, w(y) / w(c)); occupied sites weigh 0.  Per step the work is
// m_cond evaluations of one t-term sum, so a sample costs O(m_cond N^2 +
// N^3) instead of O(L N^2).
//
// Random numbers: iteration j of step t of sample s uses the Philox block
// (seed, s, t, 2 + j) (word 3 >= 2: disjoint from the sampler's stream 0
// and the DPP selection's stream 1).  Its words 0,1 pick the proposal by
// 64-bit multiply-high -- uniform over the L sites while the chain has no
// site yet or when radius == 0, else c + d with d uniform in
// [-radius, -1] u [1, radius], wrapped modulo L (a symmetric proposal) --
// and words 2,3 give u (53 bits); y is accepted when u w(c) < w(y).  A chain
// that ends without a site takes the first free site of positive weight
// (ascending), and reports NUMERICAL if there is none.
//
// One wavefront per sample; the t-term sum is split over the lanes (term i
// on lane i mod 64) and reduced by a fixed butterfly, all in float64.
#include "cx.h"
#include "ffs_internal.h"

namespace ffsk {
namespace {

template <bool C>
__device__ inline double mh_weight(const typename Cx<C>::T* U, int N, const int32_t* perm,
                                   const typename Cx<C>::T* beta, int t, int y, int lane) {
  using X = Cx<C>;
  using T = typename X::T;
  const T* row = U + (size_t)y * N;
  T acc = X::zero();
  for (int i = lane; i < t; i += 64) acc = X::fma(beta[i], row[perm[i]], acc);
  acc = wave_sum<C>(acc);
  return X::abs2(X::sub(row[perm[t]], acc));
}

__device__ inline bool occupied(const uint32_t* occ, int y) {
  return (occ[y >> 5] >> (y & 31)) & 1u;
}

template <bool C>
__global__ __launch_bounds__(256) void mh_kernel(const void* u64, const int32_t* perm_all,
                                                 const void* beta_all, int32_t* xs,
                                                 uint32_t* occ_all, int32_t* ctl,
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
  int cur = -1;
  double wc = 0.0;
  unsigned long long acc_n = 0;
  for (int j = 0; j < m_cond; ++j) {
    const Words w = philox_stream(seed, sample, (uint32_t)t, 2u + (uint32_t)j);
    const uint64_t v = ((uint64_t)w.w1 << 32) | w.w0;
    int y;
    if (radius == 0 || cur < 0) {
      y = (int)(uint64_t)(((unsigned __int128)v * (uint64_t)L) >> 64);
    } else {
      const int r = (int)(uint64_t)(((unsigned __int128)v * (uint64_t)(2 * radius)) >> 64);
      const int dlt = r < radius ? r - radius : r - radius + 1;
      y = (int)(((int64_t)cur + dlt) % L);
      if (y < 0) y += L;
    }
    const double wy = occupied(occ, y) ? 0.0 : mh_weight<C>(U, N, perm, beta, t, y, lane);
    const double u = uniform53(w);
    if (u * wc < wy) {
      cur = y;
      wc = wy;
      ++acc_n;
    }
  }
  if (cur < 0) {  // no site of positive weight met: first free one, ascending
    for (int y = 0; y < L && cur < 0; ++y)
      if (!occupied(occ, y) && mh_weight<C>(U, N, perm, beta, t, y, lane) > 0.0) cur = y;
    if (cur < 0) {
      for (int y = 0; y < L && cur < 0; ++y)
        if (!occupied(occ, y)) cur = y;
      if (lane == 0) atomicOr(&ctl[1], (int)DEV_NUMERICAL);
    }
  }
  if (lane == 0) {
    xs[(size_t)s * N + t] = cur;
    occ[cur >> 5] |= 1u << (cur & 31);
    atomicAdd(&counters[2], acc_n);
  }
}

}  // namespace

void launch_mh(const Dims& d, const Work& w, const void* u64, int S, int t, int m_cond,
               int radius, uint64_t seed, uint64_t first, hipStream_t st) {
  const dim3 grid((unsigned)((S + 3) / 4));
  if (d.cplx)
    hipLaunchKernelGGL(mh_kernel<true>, grid, dim3(256), 0, st, u64, w.perm, w.beta, w.xs, w.occ,
                       w.ctl, w.counters, S, d.L, d.L_pad, d.N, t, m_cond, radius, seed, first);
  else
    hipLaunchKernelGGL(mh_kernel<false>, grid, dim3(256), 0, st, u64, w.perm, w.beta, w.xs, w.occ,
                       w.ctl, w.counters, S, d.L, d.L_pad, d.N, t, m_cond, radius, seed, first);
}

}  // namespace ffsk
