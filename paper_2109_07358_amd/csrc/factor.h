// Per-sample float64 conditioning state and its step update (one wavefront
// per sample).  Included by the batched factor kernel and the plain path.
//
// What is computed (0-based step t; rows x_0..x_{t-1} drawn, columns
// m_0..m_{t-1} of the sample's order):
//   A_t = U[x_<t, m_<t],  c_t = U[x_<t, m_t],  beta_t = A_t^{-1} c_t,
//   Gamma_t = e_{m_t} - sum_i beta_t[i] e_{m_i},
// so that v_t(y) = U[y, :] Gamma_t = u_y^T h with h = (-beta_t, 1) normal to
// the drawn rows (Eq. (3), SI S-1).  The paper obtains h by Gaussian
// elimination extended row by row over all N columns (SI S-1); here the same
// elimination is kept as a bordered LU factorisation A_t = Lam_t R_t without
// pivoting, storing Lam_t (unit lower) and P_t = R_t^{-1} (upper) in one
// N x N column-major float64 matrix per sample:
//   element (i, j) at F[j*N + i]:  Lam(i, j) for i > j,  P(i, j) for i <= j.
// Pivoting is unnecessary because the new pivot s_t = v_t(x_t) was drawn with
// probability proportional to |s_t|^2.
//
// Step update after x_t is drawn (r = U[x_t, m_<t], a = U[x_t, m_t]):
//   s      = a - r . beta_t                  (Schur pivot = v_t(x_t))
//   ell^T  = r^T P_t                         (new row t of Lam)
//   P_{t+1} = [[P_t, -beta_t/s], [0, 1/s]]   (new column t of P)
// Solve of step t+1 (m' = m_{t+1}, c' = U[x_<=t, m']):
//   y      = Lam_t^{-1} c'[<t]               (forward substitution)
//   y_t    = c'[t] - ell . y
//   z      = P_t y
//   beta_{t+1} = [z - beta_t y_t/s ; y_t/s]
// Each step reads the t x t leading block of F once (Lam part by the forward
// substitution, P part by the fused GEMV pair) and writes O(t) words.
#pragma once

#include "cx.h"
#include "ffs_internal.h"

namespace ffsk {

// Reduce-scatter of TW per-lane values over 64 lanes: on return lane l holds
// the full 64-lane sum of value number col(l) = l * TW / 64.  Fixed butterfly
// order (deterministic).
template <bool C, int TW>
__device__ inline typename Cx<C>::T reduce_scatter(typename Cx<C>::T (&a)[TW],
                                                   int lane) {
  using X = Cx<C>;
  int n = TW;
#pragma unroll
  for (int M = 32; M >= 1; M >>= 1) {
    if (n > 1) {
      const bool up = (lane & M) != 0;
      const int h = n >> 1;
#pragma unroll
      for (int i = 0; i < TW / 2; ++i) {
        if (i < h) {
          const typename X::T lo = a[i], hi = a[i + h];
          const typename X::T send = up ? lo : hi;
          const typename X::T keep = up ? hi : lo;
          a[i] = X::add(keep, X::shfl_xor(send, M));
        }
      }
      n = h;
    } else {
      a[0] = X::add(a[0], X::shfl_xor(a[0], M));
    }
  }
  return a[0];
}

struct FacSample {
  const void* u64;   // [L][N] row-major float64 / complex128
  void* F;           // this sample's [N][N]
  int32_t* perm;     // this sample's [N]
  const int32_t* xs; // this sample's [N]
  void* beta;        // this sample's [N]
  double* logdet;    // this sample's logdet
  int32_t* status;   // device status word
  int N;
  uint64_t seed, sample;
};

// LDS needed by factor_wave: 4 vectors of N scalars + N ints.
template <bool C>
__host__ __device__ constexpr size_t factor_lds_bytes(int N) {
  return (size_t)4 * N * (C ? 16 : 8) + (size_t)N * 4;
}

// One wavefront advances one sample: absorb the draw of step t_upd (if
// t_upd >= 0) and prepare step t_solve (if t_solve >= 0).  On return the LDS
// vector `gl` holds Gamma of step t_solve (dense, length N) and pl the first
// t_solve+1 entries of the column order.
template <bool C, int TW>
__device__ void factor_wave(const FacSample& f, int t_upd, int t_solve,
                            int lane, void* lds_raw, typename Cx<C>::T** gl_out,
                            int** pl_out) {
  using X = Cx<C>;
  using T = typename X::T;
  const int N = f.N;
  T* yl = reinterpret_cast<T*>(lds_raw);
  T* rl = yl + N;
  T* zl = rl + N;
  T* ll = zl + N;
  int* pl = reinterpret_cast<int*>(ll + N);
  T* gl = rl;  // Gamma reuses r's slot once r is no longer needed
  *gl_out = gl;
  *pl_out = pl;
  const T* U = reinterpret_cast<const T*>(f.u64);
  T* F = reinterpret_cast<T*>(f.F);
  T* bv = reinterpret_cast<T*>(f.beta);

  for (int i = lane; i < N; i += 64) pl[i] = (t_upd < 0) ? i : f.perm[i];
  wave_sync();

  // ---- absorb x_t: pivot s = a - r . beta_t -------------------------------
  T s = X::one();
  const int t = t_upd;
  if (t >= 0) {
    const int xt = f.xs[t];
    const T* urow = U + (size_t)xt * N;
    T d = X::zero();
    for (int i = lane; i < t; i += 64) {
      const T r = urow[pl[i]];
      rl[i] = r;
      d = X::fma(r, bv[i], d);
    }
    d = wave_sum<C>(d);
    s = X::sub(urow[pl[t]], d);
    const double s2 = X::abs2(s);
    if (lane == 0) {
      *f.logdet += log(s2);
      if (!(s2 > 0.0) || !isfinite(s2)) atomicOr(f.status, (int)DEV_NUMERICAL);
    }
  }
  if (t_solve < 0) return;

  // ---- column draw of step t_solve (lazy Fisher-Yates) --------------------
  {
    const Words w = philox_block(f.seed, f.sample, (uint32_t)t_solve);
    const int j = fy_index(w, t_solve, N);
    const int mj = pl[j], mt = pl[t_solve];
    wave_sync();
    if (lane == 0) {
      pl[t_solve] = mj;
      pl[j] = mt;
      f.perm[t_solve] = mj;
      f.perm[j] = mt;
    }
    wave_sync();
  }
  const int mnew = pl[t_solve];

  if (t < 0) {  // first step: Gamma = e_{m_0}
    for (int i = lane; i < N; i += 64) gl[i] = X::zero();
    wave_sync();
    if (lane == 0) gl[mnew] = X::one();
    wave_sync();
    return;
  }

  // ---- c' = U[x_<=t, m'] into yl; z = 0 -----------------------------------
  for (int i = lane; i <= t; i += 64) yl[i] = U[(size_t)f.xs[i] * N + mnew];
  for (int i = lane; i < t; i += 64) zl[i] = X::zero();
  wave_sync();

  // Tiles are read with every load issued up front (addresses clamped into
  // this sample's N x N matrix, values masked afterwards), so each wavefront
  // keeps a whole tile of loads in flight instead of waiting per column.
  constexpr int DC = C ? 32 : 64;  // columns per prefetched tile
  const int Nm1 = N - 1;

  // ---- forward substitution y = Lam_t^{-1} c'[<t], by DC-column blocks -----
  for (int c0 = 0; c0 < t; c0 += DC) {
    const int ncol = min(DC, t - c0);
    // diagonal block rows c0 .. c0+DC-1 (lane -> row c0 + lane, DC <= 64)
    {
      const int row = c0 + lane;
      const bool rv = lane < DC && row < t;
      const int rowc = min(row, Nm1);
      T lv[DC];
#pragma unroll
      for (int jj = 0; jj < DC; ++jj) lv[jj] = F[(size_t)min(c0 + jj, Nm1) * N + rowc];
      T yr = rv ? yl[row] : X::zero();
#pragma unroll
      for (int jj = 0; jj < DC; ++jj) {
        if (jj < ncol) {
          const T yj = X::bcast(yr, jj);
          if (rv && lane > jj) yr = X::fnma(lv[jj], yj, yr);
        }
      }
      if (rv) yl[row] = yr;
    }
    wave_sync();
    // rows below the block: y[rows] -= Lam[rows, cols] y[cols]
    for (int r0 = c0 + DC; r0 < t; r0 += 64) {
      const int rr = r0 + lane;
      const int rrc = min(rr, Nm1);
      T lv[DC];
#pragma unroll
      for (int jj = 0; jj < DC; ++jj) lv[jj] = F[(size_t)min(c0 + jj, Nm1) * N + rrc];
      if (rr < t) {
        T acc = yl[rr];
#pragma unroll
        for (int jj = 0; jj < DC; ++jj)
          if (jj < ncol) acc = X::fnma(lv[jj], yl[c0 + jj], acc);
        yl[rr] = acc;
      }
    }
    wave_sync();
  }

  // ---- fused GEMV pair over P_t: ell = P^T r, z = P y -----------------------
  for (int c0 = 0; c0 < t; c0 += TW) {
    const int ncol = min(TW, t - c0);
    T acc[TW];
#pragma unroll
    for (int jj = 0; jj < TW; ++jj) acc[jj] = X::zero();
    const int rend = min(c0 + TW, t);
    for (int r0 = 0; r0 < rend; r0 += 64) {
      const int row = r0 + lane;
      const bool rv = row < t;
      const int rowc = min(row, Nm1);
      T pv[TW];
#pragma unroll
      for (int jj = 0; jj < TW; ++jj) pv[jj] = F[(size_t)min(c0 + jj, Nm1) * N + rowc];
      const T rr = rv ? rl[row] : X::zero();
      T zz = X::zero();
#pragma unroll
      for (int jj = 0; jj < TW; ++jj) {
        const int col = c0 + jj;
        const bool ok = rv && jj < ncol && row <= col;
        const T p = ok ? pv[jj] : X::zero();
        acc[jj] = X::fma(rr, p, acc[jj]);
        const T yc = (jj < ncol) ? yl[col] : X::zero();
        zz = X::fma(p, yc, zz);
      }
      if (rv) zl[row] = X::add(zl[row], zz);
    }
    const T v = reduce_scatter<C, TW>(acc, lane);
    const int ci = (lane * TW) / 64;
    const bool writer = (TW == 64) || ((lane & (64 / TW - 1)) == 0);
    if (writer && ci < ncol) ll[c0 + ci] = v;
  }
  wave_sync();

  // ---- assemble beta_{t+1}, extend the factor ------------------------------
  T d2 = X::zero();
  for (int i = lane; i < t; i += 64) d2 = X::fma(ll[i], yl[i], d2);
  d2 = wave_sum<C>(d2);
  const T ynew = X::sub(yl[t], d2);
  const T sinv = X::inv(s);
  const T q = X::mul(ynew, sinv);
  for (int i = lane; i < t; i += 64) {
    F[(size_t)i * N + t] = ll[i];                 // Lam(t, i)
    const T b = bv[i];
    F[(size_t)t * N + i] = X::neg(X::mul(b, sinv));  // P(i, t)
    const T bn = X::fnma(b, q, zl[i]);            // z_i - beta_i q
    bv[i] = bn;
    zl[i] = bn;
  }
  if (lane == 0) {
    F[(size_t)t * N + t] = sinv;
    bv[t] = q;
    zl[t] = q;
  }
  wave_sync();
  // Gamma of step t+1: 1 at m', -beta_{t+1}[i] at m_i (i <= t)
  for (int i = lane; i < N; i += 64) gl[i] = X::zero();
  wave_sync();
  for (int i = lane; i <= t; i += 64) gl[pl[i]] = X::neg(zl[i]);
  if (lane == 0) gl[mnew] = X::one();
  wave_sync();
}

}  // namespace ffsk
