// Block-bordered float64 conditioning state of the batched path (one
// wavefront per sample).
//
// The quantity: beta_t = A_t^{-1} c_t with A_t = U[x_<t, m_<t]
// and c_t = U[x_<t, m_t], so that Gamma_t = e_{m_t} - sum beta_t[i] e_{m_i}
// gives v_t(y) = u_y^T h (Eq. (3), SI S-1) -- but organised so that the
// large t x t factor is read once per block of BB steps instead of once per
// step.  The column order m does not depend on the draws; it is drawn whole
// by the first launch, so when x_k is drawn its entries in the columns of
// all later blocks are copied (row k of Xr) and each block boundary reads
// its 16 new columns of every earlier row contiguously.
//
// State at a block start t0 (A0 = A_{t0}):
//   Li = Lam0^{-1} (unit lower) and P = R0^{-1} (upper), A0 = Lam0 R0,
//     stored in one N x N column-major matrix F: Li(i,j) for i > j,
//     P(i,j) for i <= j;
//   E = A0^{-1} U[x_<t0, M]                       (t0 x BB, [BB][N]).
// Inside the block, after j draws x_{t0..t0+j-1}:
//   G   = U[x_{t0..t0+j-1}, m_<t0]                 ([BB][N], row r = draw r)
//   Sig = U[x_{t0..}, M] - G E                     (block Schur complement rows)
//   S_j = Sig[:j, :j] = Ls_j Rs_j kept as SLi = Ls^{-1}, SP = Rs^{-1} (BB x BB)
// Step t = t0 + j (Schur complement of the bordered system):
//   beta_bot = S_j^{-1} Sig[:j, j],  beta_top = E[:, j] - E[:, :j] beta_bot,
//   pivot s  = Sig[j, j] - Sig[j, :j] beta_bot  (= v_t(x_t)).
// Block end (t1 = t0 + BB), next columns M', C' = U[x_<t1, M']:
//   Z  = Li C'_top,  Y = P Z (= A0^{-1} C'_top),  Gn = G^T P,  Kn = Gn Li
//   (= G^T A0^{-1}),  H = C'_bot - G^T Y,  E'_bot = SP SLi H,
//   (these products run on the FP64 matrix cores),
//   E'_top = Y - E E'_bot,
//   P  gains columns [-E SP ; SP],  Li gains rows [-SLi Kn , SLi].
// All big operations are products with 16 right- or left-hand sides, so the
// t^2 factor traffic is paid once per 16 steps; per step only E and G
// (t x 16) are touched.
#pragma once

#include "factor.h"

namespace ffsk {

constexpr int BB = kFactorBlock;  // block size = MFMA N dimension (16)
static_assert(BB == 16, "the boundary products assume 16-wide MFMA tiles");

typedef double doublex4 __attribute__((ext_vector_type(4)));
// four consecutive doubles at an 8-byte aligned address
typedef double doublex4u __attribute__((ext_vector_type(4), aligned(8)));

// BB consecutive entries p[0..BB) of one lane, and the first n of them back:
// vector accesses (a lane's 128-byte row in four instructions) instead of one
// 8-byte access per entry, each of which touches 64 cache lines per
// wavefront when the lanes hold different rows.
template <bool C>
__device__ inline void load_row16(const typename Cx<C>::T* p, typename Cx<C>::T (&v)[16]) {
  if constexpr (C) {
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = p[i];
  } else {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const doublex4u x = reinterpret_cast<const doublex4u*>(p)[q];
      v[4 * q] = x.x;
      v[4 * q + 1] = x.y;
      v[4 * q + 2] = x.z;
      v[4 * q + 3] = x.w;
    }
  }
}
template <bool C>
__device__ inline void store_row16(typename Cx<C>::T* p, const typename Cx<C>::T (&v)[16], int n) {
  if constexpr (!C) {
    if (n == 16) {
#pragma unroll
      for (int q = 0; q < 4; ++q)
        reinterpret_cast<doublex4u*>(p)[q] =
            doublex4u{v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]};
      return;
    }
  }
#pragma unroll
  for (int i = 0; i < 16; ++i)
    if (i < n) p[i] = v[i];
}

// Four consecutive entries p[0..3] (p 8-byte aligned for real, 16 for complex).
template <bool C>
__device__ inline void load4(const typename Cx<C>::T* p, typename Cx<C>::T (&v)[4]) {
  if constexpr (C) {
#pragma unroll
    for (int s = 0; s < 4; ++s) v[s] = p[s];
  } else {
    const doublex4u q = *reinterpret_cast<const doublex4u*>(p);
    v[0] = q.x;
    v[1] = q.y;
    v[2] = q.z;
    v[3] = q.w;
  }
}

// FP64 16x16x4 matrix-core step on real or complex operands.  Operand layout
// (one wavefront): A[l%16][l/16], B[l/16][l%16]; accumulator register r of
// lane l holds D[l/16 + 4r][l%16].  Complex products take four real MFMAs.
template <bool C>
struct Mma;
template <>
struct Mma<false> {
  using Acc = doublex4;
  __device__ static void zero(Acc& a) { a = doublex4{0.0, 0.0, 0.0, 0.0}; }
  __device__ static void mma(Acc& acc, double a, double b) {
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
  }
  __device__ static double get(const Acc& a, int r) { return a[r]; }
  __device__ static void set(Acc& a, int r, double v) { a[r] = v; }
};
template <>
struct Mma<true> {
  struct Acc {
    doublex4 re, im;
  };
  __device__ static void zero(Acc& a) {
    a.re = doublex4{0.0, 0.0, 0.0, 0.0};
    a.im = a.re;
  }
  __device__ static void mma(Acc& acc, double2 a, double2 b) {
    acc.re = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.x, acc.re, 0, 0, 0);
    acc.re = __builtin_amdgcn_mfma_f64_16x16x4f64(-a.y, b.y, acc.re, 0, 0, 0);
    acc.im = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.y, acc.im, 0, 0, 0);
    acc.im = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, b.x, acc.im, 0, 0, 0);
  }
  __device__ static double2 get(const Acc& a, int r) { return make_double2(a.re[r], a.im[r]); }
  __device__ static void set(Acc& a, int r, double2 v) {
    a.re[r] = v.x;
    a.im[r] = v.y;
  }
};

template <bool C>
struct BlkSample {
  using T = typename Cx<C>::T;
  const T* U;        // [L][ldu] row-major
  const int32_t* cmap; // [N] column of U for each of the sample's N positions, or null (identity)
  T* F;              // [N][N]   Li / P
  T* E;              // [BB][N]
  T* Z;              // [N][BB]  scratch: C', then Z, then Y
  T* G;              // [BB][N]  G(k, r) = U[x_{t0+r}, m_k] at r * N + k
  T* Gn;             // [N][BB]  scratch: G^T P
  T* Kn;             // [N][BB]  scratch: G^T A0^{-1}
  T* Sg;             // [BB][BB] Sig rows, (r, i) at r*BB + i
  T* SLi;            // [BB][BB] Ls^{-1}, (r, c) at r*BB + c
  T* SP;             // [BB][BB] Rs^{-1}, (r, c) at r*BB + c
  T* Xr;             // [N][N]   Xr(k, c) = U[x_k, m_c] for c >= (block of k) + BB
  T* beta;           // [N]
  int32_t* perm;     // [N]
  const int32_t* xs; // [N]
  double* logdet;
  int32_t* status;
  int N, n_steps, ldu;
  uint64_t seed, sample;
};

// Column of U behind position c of the sample's column order.
template <bool C>
__device__ inline int ucol(const BlkSample<C>& f, int c) {
  return f.cmap ? f.cmap[c] : c;
}

// Per-sample element count of the state (in units of T).
__host__ __device__ constexpr size_t blk_state_elems(int N) {
  return (size_t)2 * N * N + (size_t)5 * BB * N + (size_t)3 * BB * BB;
}

// LDS of blk_wave: gam[N], three BB x BB matrices and four BB vectors that
// every step uses, pl[N] ints, then (block-closing launches only) three more
// BB x BB matrices.  Regular launches leave the last part out, which lets
// more wavefronts share a CU.
template <bool C>
__host__ __device__ constexpr size_t blk_lds_head_bytes(int N) {
  return ((size_t)N * (C ? 16 : 8) + (size_t)3 * BB * BB * (C ? 16 : 8) +
          (size_t)4 * BB * (C ? 16 : 8) + (size_t)N * 4 + 15) / 16 * 16;
}
template <bool C, bool BND = true>
__host__ __device__ constexpr size_t blk_lds_bytes(int N) {
  return blk_lds_head_bytes<C>(N) + (BND ? (size_t)3 * BB * BB * (C ? 16 : 8) : 0);
}

// Element (row, col) of the N x N column-major factor matrix.
template <bool C>
__device__ inline typename Cx<C>::T F_at(const BlkSample<C>& f, int col, int row) {
  return f.F[(size_t)col * f.N + row];
}
template <bool C>
__device__ inline typename Cx<C>::T& F_ref(const BlkSample<C>& f, int col, int row) {
  return f.F[(size_t)col * f.N + row];
}

// Global stores of one lane become visible to the other lanes of the
// wavefront (the only readers) after this (workgroup = one wavefront here).
__device__ inline void lane_fence() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
}

// BND selects the instantiation for launches that close a block (the host
// knows which steps those are); the regular instantiation carries none of
// the boundary code, which keeps its register footprint small.
template <bool C, bool BND>
__device__ void blk_wave(const BlkSample<C>& f, int t_upd, int t_solve,
                         int lane, void* lds_raw, typename Cx<C>::T** gam_out) {
  using X = Cx<C>;
  using T = typename X::T;
  const int N = f.N, Nm1 = N - 1;
  char* p = reinterpret_cast<char*>(lds_raw);
  T* gam = reinterpret_cast<T*>(p);            p += (size_t)N * sizeof(T);
  T* sgl = reinterpret_cast<T*>(p);            p += BB * BB * sizeof(T);
  T* sli = reinterpret_cast<T*>(p);            p += BB * BB * sizeof(T);
  T* spl = reinterpret_cast<T*>(p);            p += BB * BB * sizeof(T);
  T* vec = reinterpret_cast<T*>(p);            p += 4 * BB * sizeof(T);
  int* pl = reinterpret_cast<int*>(p);
  p = reinterpret_cast<char*>(lds_raw) + blk_lds_head_bytes<C>(N);
  T* hl = reinterpret_cast<T*>(p);             p += BB * BB * sizeof(T);  // BND only
  T* ul = reinterpret_cast<T*>(p);             p += BB * BB * sizeof(T);  // BND only
  T* ebl = reinterpret_cast<T*>(p);                                       // BND only
  T* bbl = vec;           // beta_bot
  T* lsl = vec + BB;      // ell_s
  T* uvl = vec + 2 * BB;  // Ls^{-1} Sig[:, j]
  *gam_out = gam;

  for (int i = lane; i < N; i += 64) pl[i] = (t_upd < 0) ? i : f.perm[i];
  for (int i = lane; i < BB * BB; i += 64) {
    if (t_upd >= 0) {
      sgl[i] = f.Sg[i];
      sli[i] = f.SLi[i];
      spl[i] = f.SP[i];
    }
  }
  wave_sync();

  int t0;
  if (t_upd < 0) {
    // The whole column order at once: the Fisher-Yates index of every
    // position (one Philox block each, in parallel; gam is free until the
    // solve below), then the swaps in order.  Position t ends as the lazy
    // draw at step t would leave it, so each row's later columns are known
    // when the row is drawn.
    t0 = 0;
    int* jt = reinterpret_cast<int*>(gam);
    for (int t = lane; t < N; t += 64)
      jt[t] = fy_index(philox_block(f.seed, f.sample, (uint32_t)t), t, N);
    wave_sync();
    if (lane == 0)
      for (int t = 0; t < N; ++t) {
        const int j = jt[t];
        const int mj = pl[j];
        pl[j] = pl[t];
        pl[t] = mj;
      }
    wave_sync();
    for (int i = lane; i < N; i += 64) f.perm[i] = pl[i];
  } else {
    // ================= absorb x_t (t = t0 + j) =================
    const int t = t_upd;
    t0 = (t / BB) * BB;
    const int j = t - t0;
    // Blocks are cut from N alone (not from the number of steps run), so a
    // marginal run is bit-for-bit a prefix of the full run: columns past
    // the last step only fill unused columns of E.
    const int nb = min(BB, N - t0);
    const int xt = f.xs[t];
    const T* urow = f.U + (size_t)xt * f.ldu;
    // w = E[:nb, :t0] g, g = U[x_t, m_<t0]; G[:, j] = g.  Loads that do not
    // depend on the sum (the row entries of the new block columns, beta) are
    // issued first; real operands take two 64-wide chunks of k per round
    // trip, accumulated in the same k order as one chunk at a time.
    const int ib = lane >> 2;
    const bool sig_lane = (lane & 3) == 0 && ib < nb;
    const T ublk = sig_lane ? urow[ucol(f, pl[t0 + ib])] : X::zero();
    const T bet_j = (lane < j) ? f.beta[t0 + lane] : X::zero();
    T acc[BB];
#pragma unroll
    for (int i = 0; i < BB; ++i) acc[i] = X::zero();
    constexpr int CH = C ? 1 : 2;
    for (int k0 = 0; k0 < t0; k0 += 64 * CH) {
      T ev[CH][BB], g[CH];
      bool ok[CH];
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        const int k = k0 + 64 * c + lane;
        ok[c] = k < t0;
        if (c == 0 || k0 + 64 * c < t0) {
          const int kc = min(k, Nm1);
          // rows k >= t0 of E are not needed: not loaded
#pragma unroll
          for (int i = 0; i < BB; ++i) ev[c][i] = ok[c] ? f.E[(size_t)i * N + k] : X::zero();
          g[c] = ok[c] ? urow[ucol(f, pl[kc])] : X::zero();
          if (ok[c]) f.G[(size_t)j * N + k] = g[c];
        }
      }
#pragma unroll
      for (int c = 0; c < CH; ++c)
        if (c == 0 || k0 + 64 * c < t0) {
#pragma unroll
          for (int i = 0; i < BB; ++i) acc[i] = X::fma(g[c], ok[c] ? ev[c][i] : X::zero(), acc[i]);
        }
    }
    const T wv = reduce_scatter<C, BB>(acc, lane);
    if (sig_lane) sgl[j * BB + ib] = X::sub(ublk, wv);
    // the row's entries in the columns of later blocks, read by the block
    // boundaries that need them
    for (int c = t0 + BB + lane; c < N; c += 64)
      f.Xr[(size_t)t * N + c] = urow[ucol(f, pl[c])];
    wave_sync();
    // pivot s = Sig[j, j] - Sig[j, :j] beta_bot
    T d = X::zero();
    if (lane < j) d = X::mul(sgl[j * BB + lane], bet_j);
    d = wave_sum<C>(d);
    const T s = X::sub(sgl[j * BB + j], d);
    const double s2 = X::abs2(s);
    if (lane == 0) {
      *f.logdet += log(s2);
      if (!(s2 > 0.0) || !isfinite(s2)) atomicOr(f.status, (int)DEV_NUMERICAL);
    }
    const T sinv = X::inv(s);
    // bordered inverse factors of S_{j+1}: ell_s = Sig[j,:j] SP; new SLi row;
    // new SP column [-beta_bot/s ; 1/s]
    if (lane < j) {
      T a = X::zero();
      for (int i = 0; i <= lane; ++i) a = X::fma(sgl[j * BB + i], spl[i * BB + lane], a);
      lsl[lane] = a;
    }
    wave_sync();
    if (lane < j) {
      T a = lsl[lane];
      for (int r = lane + 1; r < j; ++r) a = X::fma(lsl[r], sli[r * BB + lane], a);
      sli[j * BB + lane] = X::neg(a);
      spl[lane * BB + j] = X::neg(X::mul(bet_j, sinv));
    }
    if (lane == 0) {
      sli[j * BB + j] = X::one();
      spl[j * BB + j] = sinv;
    }
    wave_sync();
    // persist the small state
    if (lane < BB) {
      f.Sg[j * BB + lane] = sgl[j * BB + lane];
      f.SLi[j * BB + lane] = sli[j * BB + lane];
      f.SP[lane * BB + j] = spl[lane * BB + j];
    }
    if (t_solve < 0) return;

    if (BND && j == nb - 1) {
      // ================= block boundary t0 -> t1 =================
      const int t1 = t0 + nb;
      const int nb2 = min(BB, N - t1);
      // C' = U[x_<t1, M'] into Z, from the rows' stored later columns (four
      // rows of 16 per instruction, coalesced)
      lane_fence();
      {
        const int i = lane & 15;
        for (int k0 = 0; k0 < t1; k0 += 16) {
          T v[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int k = k0 + 4 * q + (lane >> 4);
            v[q] = (k < t1 && i < nb2) ? f.Xr[(size_t)k * N + t1 + i] : X::zero();
          }
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int k = k0 + 4 * q + (lane >> 4);
            if (k < t1) f.Z[(size_t)k * BB + i] = v[q];
          }
        }
      }
      lane_fence();
      // Passes A-D and H run on the FP64 matrix cores (v_mfma_f64_16x16x4f64):
      // each wavefront computes a 64-row x 16-column block as four 16 x 16
      // tiles; operands come straight from coalesced global loads.
      using M = Mma<C>;
      auto ld_rows = [&](typename M::Acc (&acc)[4], const T* src, int r0, int nrows) {
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = r0 + 16 * mt + (lane >> 4) + 4 * r;
            const T v = (row < nrows) ? src[(size_t)min(row, Nm1) * BB + (lane & 15)] : X::zero();
            M::set(acc[mt], r, v);
          }
      };
      auto st_rows = [&](const typename M::Acc (&acc)[4], T* dst, int r0, int nrows) {
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = r0 + 16 * mt + (lane >> 4) + 4 * r;
            if (row < nrows) dst[(size_t)row * BB + (lane & 15)] = M::get(acc[mt], r);
          }
      };
      // B element accessor of an [N][BB] row-major panel
      auto rows_of = [&](const T* Bm) {
        return [=](int k) { return Bm[(size_t)k * BB + (lane & 15)]; };
      };
      // acc[mt] += A(rows r0.., k) B(k, 0..15) for k in [kbeg, kend);
      // a_at(row, k) returns the (masked) A element -- masked entries are
      // not loaded, so the other triangle and the rows past t0 of a partial
      // 64-row block cost no memory traffic -- and b_at(k) this lane's B
      // element of row k (k clamped to [0, N)).
      auto mma_rows = [&](typename M::Acc (&acc)[4], int r0, int kbeg, int kend,
                          auto a_at, auto b_at) {
        for (int kb = kbeg; kb < kend; kb += 16) {
          T av[4][4], bv[4];
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            const int k = kb + 4 * s + (lane >> 4);
            bv[s] = (k < kend) ? b_at(min(k, Nm1)) : X::zero();
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) av[s][mt] = a_at(r0 + 16 * mt + (lane & 15), k, k < kend);
          }
#pragma unroll
          for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) M::mma(acc[mt], av[s][mt], bv[s]);
        }
      };
      // Same product for an A read along its rows (A(row, k) = arow(row)[k],
      // contiguous in k).  Lane group g = lane / 16 takes k = kb + 4g + s for
      // MFMA s = 0..3 (the same k in both operands, so each MFMA still sums
      // four k and the 16-wide group is covered), which lets a lane read its
      // four A entries -- and a B panel that is also contiguous in k -- with
      // one vector load instead of four row segments of 32 bytes.  need(row,
      // k) is the A mask; masked entries load nothing.
      auto mma_rows_t = [&](typename M::Acc (&acc)[4], int r0, int kbeg, int kend,
                            auto need, auto arow, auto b_load) {
        for (int kb = kbeg; kb < kend; kb += 16) {
          const int kq = kb + 4 * (lane >> 4);
          T av[4][4], bv[4];
          b_load(kq, kend, bv);
#pragma unroll
          for (int mt = 0; mt < 4; ++mt) {
            const int row = r0 + 16 * mt + (lane & 15);
            bool m[4], any = false;
#pragma unroll
            for (int s = 0; s < 4; ++s) {
              m[s] = kq + s < kend && row < t0 && need(row, kq + s);
              any = any || m[s];
            }
            T v[4] = {X::zero(), X::zero(), X::zero(), X::zero()};
            if (any) load4<C>(arow(row) + kq, v);
#pragma unroll
            for (int s = 0; s < 4; ++s) av[s][mt] = m[s] ? v[s] : X::zero();
          }
#pragma unroll
          for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) M::mma(acc[mt], av[s][mt], bv[s]);
        }
      };
      auto frow = [&](int row) { return f.F + (size_t)row * N; };
      // pass A: Z[:t0] = Li Z[:t0] (unit lower; descending row blocks, in place)
      for (int k0 = ((t0 - 1) / 64) * 64; k0 >= 0 && t0 > 0; k0 -= 64) {
        typename M::Acc acc[4];
        ld_rows(acc, f.Z, k0, t0);
        mma_rows(acc, k0, 0, min(k0 + 64, t0),
                 [&](int row, int k, bool kin) -> T {
                   return (kin && row < t0 && k < row) ? F_at(f, k, row) : X::zero();
                 }, rows_of(f.Z));
        lane_fence();
        st_rows(acc, f.Z, k0, t0);
        lane_fence();
      }
      // pass B: Z[:t0] = P Z[:t0] (upper; ascending row blocks, in place)
      for (int i0 = 0; i0 < t0; i0 += 64) {
        typename M::Acc acc[4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) M::zero(acc[mt]);
        mma_rows(acc, i0, i0, t0,
                 [&](int row, int k, bool kin) -> T {
                   return (kin && row < t0 && k >= row) ? F_at(f, k, row) : X::zero();
                 }, rows_of(f.Z));
        lane_fence();
        st_rows(acc, f.Z, i0, t0);
        lane_fence();
      }
      // pass C: Gn[c][r] = sum_{i<=c} P[i][c] G[i][r]
      for (int c0 = 0; c0 < t0; c0 += 64) {
        typename M::Acc acc[4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) M::zero(acc[mt]);
        const int kend = min(c0 + 64, t0);
        mma_rows_t(acc, c0, 0, kend, [](int row, int k) { return k <= row; }, frow,
                   [&](int kq, int ke, T (&bv)[4]) {  // G(r = lane % 16, k), contiguous in k
                     if (kq < ke) {
                       load4<C>(f.G + (size_t)(lane & 15) * N + kq, bv);
                     } else {
#pragma unroll
                       for (int s = 0; s < 4; ++s) bv[s] = X::zero();
                     }
                   });
        st_rows(acc, f.Gn, c0, t0);
      }
      lane_fence();
      // pass D: Kn[c'][r] = Gn[c'][r] + sum_{c>c'} Li[c][c'] Gn[c][r]
      for (int c0 = 0; c0 < t0; c0 += 64) {
        typename M::Acc acc[4];
        ld_rows(acc, f.Gn, c0, t0);
        mma_rows_t(acc, c0, c0, t0, [](int row, int k) { return k > row; }, frow,
                   [&](int kq, int ke, T (&bv)[4]) {  // Gn(k, r = lane % 16)
#pragma unroll
                     for (int s = 0; s < 4; ++s)
                       bv[s] = kq + s < ke ? f.Gn[(size_t)(kq + s) * BB + (lane & 15)] : X::zero();
                   });
        st_rows(acc, f.Kn, c0, t0);
      }
      lane_fence();
      // H = C'_bot - G^T Y  (nb x nb2), one 16 x 16 tile over k < t0
      {
        typename M::Acc h;
        M::zero(h);
        for (int kb = 0; kb < t0; kb += 16) {
          T av[4], bv[4];
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            const int k = kb + 4 * s + (lane >> 4);
            const bool kin = k < t0;
            const int kc = min(k, Nm1);
            av[s] = kin ? f.G[(size_t)(lane & 15) * N + kc] : X::zero();
            bv[s] = kin ? f.Z[(size_t)kc * BB + (lane & 15)] : X::zero();
          }
#pragma unroll
          for (int s = 0; s < 4; ++s) M::mma(h, av[s], bv[s]);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int rr = (lane >> 4) + 4 * r, i = lane & 15;
          const T cbv = f.Z[(size_t)min(t0 + rr, Nm1) * BB + i];
          hl[rr * BB + i] = (rr < nb && i < nb2) ? X::sub(cbv, M::get(h, r)) : X::zero();
        }
      }
      wave_sync();
      // E'_bot = SP (SLi H): two small triangular products
      for (int e = lane; e < BB * BB; e += 64) {
        const int r = e / BB, i = e % BB;
        T a = X::zero();
        for (int r2 = 0; r2 <= r; ++r2)
          a = X::fma(r2 == r ? X::one() : sli[r * BB + r2], hl[r2 * BB + i], a);
        ul[e] = (r < nb) ? a : X::zero();
      }
      wave_sync();
      for (int e = lane; e < BB * BB; e += 64) {
        const int r = e / BB, i = e % BB;
        T a = X::zero();
        for (int r2 = r; r2 < nb; ++r2) a = X::fma(spl[r * BB + r2], ul[r2 * BB + i], a);
        ebl[e] = (r < nb) ? a : X::zero();
      }
      wave_sync();
      // rows k < t0: new P columns -E SP and E'_top = Y - E E'_bot
      for (int k0 = 0; k0 < t0; k0 += 64) {
        const int k = k0 + lane;
        if (k < t0) {
          T eo[BB], y[BB];
#pragma unroll
          for (int r = 0; r < BB; ++r) eo[r] = (r < nb) ? f.E[(size_t)r * N + k] : X::zero();
          load_row16<C>(f.Z + (size_t)k * BB, y);
#pragma unroll
          for (int c = 0; c < BB; ++c) {  // static indices keep eo in registers
            T a = X::zero();
#pragma unroll
            for (int r = 0; r < BB; ++r)
              if (r <= c) a = X::fma(eo[r], spl[r * BB + c], a);
            if (c < nb) F_ref(f, t0 + c, k) = X::neg(a);
          }
#pragma unroll
          for (int i = 0; i < BB; ++i) {
            T a = y[i];
#pragma unroll
            for (int r = 0; r < BB; ++r) a = X::fnma(eo[r], ebl[r * BB + i], a);
            if (i < nb2) f.E[(size_t)i * N + k] = a;
          }
        }
      }
      // columns c < t0: new Li rows -SLi Kn
      for (int c0 = 0; c0 < t0; c0 += 64) {
        const int c = c0 + lane;
        if (c < t0) {
          T kn[BB];
          load_row16<C>(f.Kn + (size_t)c * BB, kn);
          if constexpr (!C) {  // the row F(t0 + r, c), r < nb, as vector stores
            T li[BB];
#pragma unroll
            for (int r = 0; r < BB; ++r) {  // static indices keep kn in registers
              T a = kn[r];
#pragma unroll
              for (int r2 = 0; r2 < BB; ++r2)
                if (r2 < r) a = X::fma(sli[r * BB + r2], kn[r2], a);
              li[r] = X::neg(a);
            }
            store_row16<C>(&F_ref(f, c, t0), li, nb);
          } else {  // complex: a second 16-entry array would spill
#pragma unroll
            for (int r = 0; r < BB; ++r) {
              T a = kn[r];
#pragma unroll
              for (int r2 = 0; r2 < BB; ++r2)
                if (r2 < r) a = X::fma(sli[r * BB + r2], kn[r2], a);
              if (r < nb) F_ref(f, c, t0 + r) = X::neg(a);
            }
          }
        }
      }
      // diagonal block and E'_bot rows
      for (int e = lane; e < BB * BB; e += 64) {
        const int r = e / BB, c = e % BB;
        if (r < nb && c < nb) F_ref(f, t0 + c, t0 + r) = (r <= c) ? spl[r * BB + c] : sli[r * BB + c];
        const int i = c;
        if (r < nb && i < nb2) f.E[(size_t)i * N + t0 + r] = ebl[r * BB + i];
      }
      lane_fence();
      t0 = t1;
    }
  }

  // ================= prepare step ts = t0 + j =================
  const int ts = t_solve;
  const int j = ts - t0;
  if (j > 0) {
    // beta_bot = SP_j SLi_j Sig[:j, j]
    if (lane < j) {
      T a = X::zero();
      for (int r2 = 0; r2 <= lane; ++r2)
        a = X::fma(r2 == lane ? X::one() : sli[lane * BB + r2], sgl[r2 * BB + j], a);
      uvl[lane] = a;
    }
    wave_sync();
    if (lane < j) {
      T a = X::zero();
      for (int r = lane; r < j; ++r) a = X::fma(spl[lane * BB + r], uvl[r], a);
      bbl[lane] = a;
    }
    wave_sync();
  }
  for (int i = lane; i < N; i += 64) gam[i] = X::zero();
  wave_sync();
  constexpr int CHP = C ? 1 : 2;  // 64-wide chunks of k per round trip
  // beta_top needs columns 0..j of E (rows k < t0) only; nothing else is
  // loaded
  for (int k0 = 0; k0 < t0; k0 += 64 * CHP) {
    T ev[CHP][BB];
#pragma unroll
    for (int c = 0; c < CHP; ++c)
      if (c == 0 || k0 + 64 * c < t0) {
        const int k = k0 + 64 * c + lane;
#pragma unroll
        for (int i = 0; i < BB; ++i)
          ev[c][i] = (i <= j && k < t0) ? f.E[(size_t)i * N + k] : X::zero();
      }
#pragma unroll
    for (int c = 0; c < CHP; ++c) {
      const int k = k0 + 64 * c + lane;
      if (k < t0) {
        T a = X::zero();
#pragma unroll
        for (int i = 0; i < BB; ++i)
          if (i == j) a = ev[c][i];
#pragma unroll
        for (int i = 0; i < BB; ++i)
          if (i < j) a = X::fnma(ev[c][i], bbl[i], a);
        f.beta[k] = a;
        gam[pl[k]] = X::neg(a);
      }
    }
  }
  if (lane < j) {
    f.beta[t0 + lane] = bbl[lane];
    gam[pl[t0 + lane]] = X::neg(bbl[lane]);
  }
  if (lane == 0) gam[pl[ts]] = X::one();
  wave_sync();
}

}  // namespace ffsk
