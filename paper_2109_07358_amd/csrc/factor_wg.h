// Workgroup-parallel float64 conditioning update of the plain path (one
// sample per workgroup, all wavefronts working on it).
//
// The quantity: beta_t = A_t^{-1} c_t with A_t = U[x_<t, m_<t],
// c_t = U[x_<t, m_t], so that Gamma_t = e_{m_t} - sum beta_t[i] e_{m_i} gives
// v_t(y) = u_y^T h (Eq. (3), SI S-1), with the elimination kept as the
// inverse factors of A_t = Lam R (Lam unit lower): Li = Lam^{-1} and
// P = R^{-1}, so that every product of a step is a set of independent dot
// products with no sequential substitution.  Each factor is stored twice,
// column-major and row-major, so that every dot product reads contiguous
// memory.
//
// Absorbing the draw x_u of step u (r = U[x_u, m_<u], a = U[x_u, m_u]):
//   s = a - r . beta_u                         (pivot = v_u(x_u))
//   ell^T = r^T P,   gamma^T = ell^T Li        (row u of Lam, Li)
//   Li gains row u: -gamma^T (unit diagonal);  P gains column u: -beta_u/s, 1/s
// Solving step t = u + 1 (column m' = m_t, c' = U[x_<=u, m']):
//   y_<u = Li c'_<u,  y_u = c'_u - gamma . c'_<u,  z = P y_<u
//   beta_t = [z - beta_u y_u / s ; y_u / s]
// The four t x t triangular products (ell, gamma, y, z) read 2 t^2 words per
// step; they are split over the wavefronts in tiles of DT outputs, each
// tile's sums formed inside one wavefront in a fixed order.
#pragma once

#include "cx.h"
#include "factor.h"
#include "ffs_internal.h"

namespace ffsk {

constexpr int DT = 8;  // outputs per dot-product tile

template <bool C>
struct WgState {
  const typename Cx<C>::T* u64;  // [L][N] row-major
  typename Cx<C>::T* LiC;        // N x N, Li(i, j) at [j*N + i]
  typename Cx<C>::T* LiR;        // N x N, Li(i, j) at [i*N + j]
  typename Cx<C>::T* PC;         // N x N, P(i, j) at [j*N + i]
  typename Cx<C>::T* PR;         // N x N, P(i, j) at [i*N + j]
  const int32_t* xs;             // drawn sites [N]
  double* logdet;
  int32_t* status;
  int N;
  uint64_t seed, sample;
};

// LDS of factor_wg: six vectors of N scalars, 16 reduction slots, the column
// order pl[N].
template <bool C>
__host__ __device__ constexpr size_t wg_lds_bytes(int N) {
  return (size_t)(6 * N + 16) * (C ? 16 : 8) + (size_t)N * 4;
}

template <bool C>
struct WgLds {
  typename Cx<C>::T *bet, *rr, *cc, *ll, *gg, *yy, *red;
  int* pl;
  __device__ WgLds(char* lds, int N) {
    using T = typename Cx<C>::T;
    bet = reinterpret_cast<T*>(lds);
    rr = bet + N;
    cc = rr + N;
    ll = cc + N;
    gg = ll + N;
    yy = gg + N;
    red = yy + N;
    pl = reinterpret_cast<int*>(red + 16);
  }
};

// out(o, sum_{k in [lo(o), hi(o))} row(o)[k] * v[k]) for o in [0, n_out):
// tiles of DT consecutive outputs, tile k of the concatenated job list taken
// by wavefront k mod nw.  Within a tile a lane visits k = kb + lane in
// ascending kb, then reduce_scatter combines the lanes in a fixed butterfly.
template <bool C, class Row, class Lo, class Hi, class Out>
__device__ inline void dot_tile(int o0, int n_out, int N, Row row, Lo lo, Hi hi,
                                const typename Cx<C>::T* v, Out out, int lane) {
  using X = Cx<C>;
  using T = typename X::T;
  const int nout = min(DT, n_out - o0);
  int klo = N, khi = 0;
#pragma unroll
  for (int d = 0; d < DT; ++d)
    if (d < nout) {
      klo = min(klo, lo(o0 + d));
      khi = max(khi, hi(o0 + d));
    }
  T acc[DT];
#pragma unroll
  for (int d = 0; d < DT; ++d) acc[d] = X::zero();
  for (int kb = klo; kb < khi; kb += 64) {
    const int k = kb + lane;
    const int kc = min(k, N - 1);
    const T vk = (k < khi) ? v[kc] : X::zero();
    T m[DT];
#pragma unroll
    for (int d = 0; d < DT; ++d) {
      const int o = min(o0 + d, n_out - 1);
      m[d] = row(o)[kc];
    }
#pragma unroll
    for (int d = 0; d < DT; ++d) {
      const int o = o0 + d;
      const bool in = d < nout && k >= lo(min(o, n_out - 1)) && k < hi(min(o, n_out - 1));
      acc[d] = X::fma(in ? m[d] : X::zero(), vk, acc[d]);
    }
  }
  const T r = reduce_scatter<C, DT>(acc, lane);
  const int d = (lane * DT) / 64;
  if ((lane & (64 / DT - 1)) == 0 && d < nout) out(o0 + d, r);
}

// One step of the conditioning state, called by all PT threads of the
// workgroup: absorb x_{t_upd} (t_upd >= 0) and prepare step t_solve (>= 0).
// On return bet[0..t_solve) holds beta of step t_solve and pl the column
// order (pl[t_solve] = m_t).  Ends with a workgroup barrier.
template <bool C>
__device__ void factor_wg(const WgState<C>& f, int t_upd, int t_solve,
                          const WgLds<C>& s, int tid, int nthreads) {
  using X = Cx<C>;
  using T = typename X::T;
  const int N = f.N;
  const int wave = tid >> 6, lane = tid & 63, nw = nthreads >> 6;
  const int u = t_upd;

  // ---- column draw of step t_solve (lazy Fisher-Yates) ---------------------
  if (tid == 0 && t_solve >= 0) {
    const Words w = philox_block(f.seed, f.sample, (uint32_t)t_solve);
    const int j = fy_index(w, t_solve, N);
    const int mj = s.pl[j];
    s.pl[j] = s.pl[t_solve];
    s.pl[t_solve] = mj;
  }
  __syncthreads();
  if (u < 0) return;  // first step: Gamma = e_{m_0}, nothing to factor
  const int mnew = t_solve >= 0 ? s.pl[t_solve] : 0;

  // ---- gathers: r, c'; partial dot r . beta --------------------------------
  const int xu = f.xs[u];
  const T* urow = f.u64 + (size_t)xu * N;
  T part = X::zero();
  for (int i = tid; i < u; i += nthreads) {
    const T r = urow[s.pl[i]];
    s.rr[i] = r;
    part = X::fma(r, s.bet[i], part);
  }
  if (t_solve >= 0)
    for (int i = tid; i <= u; i += nthreads) s.cc[i] = f.u64[(size_t)f.xs[i] * N + mnew];
  part = wave_sum<C>(part);
  if (lane == 0) s.red[wave] = part;
  __syncthreads();
  T dot = X::zero();
  for (int w = 0; w < nw; ++w) dot = X::add(dot, s.red[w]);
  const T piv = X::sub(urow[s.pl[u]], dot);
  if (tid == 0) {
    const double s2 = X::abs2(piv);
    *f.logdet += log(s2);
    if (!(s2 > 0.0) || !isfinite(s2)) atomicOr(f.status, (int)DEV_NUMERICAL);
  }
  if (t_solve < 0) {
    __syncthreads();
    return;
  }
  const T sinv = X::inv(piv);

  // ---- ell^T = r^T P (columns of P) ----------------------------------------
  const int nt = (u + DT - 1) / DT;
  for (int k = wave; k < nt; k += nw)
    dot_tile<C>(
        k * DT, u, N, [&](int o) { return f.PC + (size_t)o * N; }, [](int) { return 0; },
        [](int o) { return o + 1; }, s.rr, [&](int o, T v) { s.ll[o] = v; }, lane);
  __syncthreads();

  // ---- gamma^T = ell^T Li (columns of Li) and y_<u = Li c'_<u (rows) --------
  for (int k = wave; k < 2 * nt; k += nw) {
    if (k < nt)
      dot_tile<C>(
          k * DT, u, N, [&](int o) { return f.LiC + (size_t)o * N; },
          [](int o) { return o + 1; }, [&](int) { return u; }, s.ll,
          [&](int o, T v) { s.gg[o] = X::add(s.ll[o], v); }, lane);
    else
      dot_tile<C>(
          (k - nt) * DT, u, N, [&](int o) { return f.LiR + (size_t)o * N; },
          [](int) { return 0; }, [](int o) { return o; }, s.cc,
          [&](int o, T v) { s.yy[o] = X::add(s.cc[o], v); }, lane);
  }
  __syncthreads();

  // ---- extend the factors; y_u = c'_u - gamma . c'_<u ------------------------
  part = X::zero();
  for (int i = tid; i < u; i += nthreads) {
    const T g = X::neg(s.gg[i]);
    f.LiR[(size_t)u * N + i] = g;
    f.LiC[(size_t)i * N + u] = g;
    const T pc = X::neg(X::mul(s.bet[i], sinv));
    f.PC[(size_t)u * N + i] = pc;
    f.PR[(size_t)i * N + u] = pc;
    part = X::fma(s.gg[i], s.cc[i], part);
  }
  if (tid == 0) {
    f.PC[(size_t)u * N + u] = sinv;
    f.PR[(size_t)u * N + u] = sinv;
  }
  part = wave_sum<C>(part);
  if (lane == 0) s.red[8 + wave] = part;
  __syncthreads();
  T gc = X::zero();
  for (int w = 0; w < nw; ++w) gc = X::add(gc, s.red[8 + w]);
  const T yu = X::sub(s.cc[u], gc);

  // ---- z = P y_<u (rows of P, columns < u) ---------------------------------
  for (int k = wave; k < nt; k += nw)
    dot_tile<C>(
        k * DT, u, N, [&](int o) { return f.PR + (size_t)o * N; }, [](int o) { return o; },
        [&](int) { return u; }, s.yy, [&](int o, T v) { s.rr[o] = v; }, lane);
  __syncthreads();

  // ---- beta of step t = u + 1 ----------------------------------------------
  const T q = X::mul(yu, sinv);
  for (int i = tid; i < u; i += nthreads) s.bet[i] = X::fnma(s.bet[i], q, s.rr[i]);
  if (tid == 0) s.bet[u] = q;
  __syncthreads();
}

}  // namespace ffsk
