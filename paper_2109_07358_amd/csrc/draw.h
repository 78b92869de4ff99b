// Inverse-CDF draw of the batched path (one wavefront per sample) and the
// float64 redraw of a flagged draw; shared by the separate draw launches and
// the fused draw + factor launch of deferred resolution.
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
// that scale times a safety factor fixed per bulk mode.
//
// A flagged draw is resolved from float64 weights V = U Gamma of its step
// (the float64 product of k_draw.hip) with the same u, either per step --
// the flagging wavefront queues it and lays out its dense float64 Gamma,
// and the next factor launch redraws it before absorbing the draw -- or
// deferred: the draw keeps its float32 site and is recorded (Gamma and the
// occupancy at that step); at the end of the call each record's float64
// site is formed the same way, and a sample whose site moved is replayed
// with per-step resolution.  Both give the same sites: a sample none of
// whose recorded draws moved followed the trajectory per-step resolution
// would have taken.
#pragma once

#include "args.h"
#include "cx.h"
#include "ffs_internal.h"

namespace ffsk {

// Float64 site of a flagged draw at step t of Philox sample `sample`, with
// the draw's u, from its float64 weights wr[0..L_pad) and 64-site chunk sums
// cs[0..L_pad/64).  The running sums are formed in fixed-order levels, as in
// the float32 draw:
// lane l owns q = ceil(nch / 64) consecutive chunks and sums them in order;
// chunk bounds are those lane totals added in ascending lane order, then the
// owner's chunks in order (its last chunk ends at the next lane's bound),
// then the chosen chunk's sites in order (the last site takes the chunk
// end).  The scans run on lane 0 (a redraw is rare; the factor kernel's
// register budget is not spent on it); lds holds the 64 lane totals and the
// chosen chunk (1 KB, before the factor update uses it).  Returns the site
// on every lane, or -1 when there is no float64 mass.
__device__ inline int redraw_site(const double* cs, const double* wr, int L_pad, uint64_t seed,
                                  uint64_t sample, int t, int lane, char* lds) {
  double* shp = reinterpret_cast<double*>(lds);  // [64] lane totals
  double* wl = shp + 64;                          // [RCHUNK] chosen chunk
  int* sc = reinterpret_cast<int*>(wl + RCHUNK);  // chosen chunk
  double* sv = reinterpret_cast<double*>(sc + 2); // its start and end, target
  const int nch = L_pad / RCHUNK;
  const int q = (nch + 63) / 64;
  {
    const int c0 = lane * q, cn = max(0, min(q, nch - c0));
    double P = 0.0;
    #pragma unroll 1
    for (int j = 0; j < cn; ++j) P += cs[c0 + j];
    shp[lane] = P;
  }
  wave_sync();
  if (lane == 0) {
    // few live values here: the factor kernel's register budget is set by
    // its largest live range, and this branch is inlined into it
    double T64 = 0.0;
    #pragma unroll 1
    for (int l = 0; l < 64; ++l) T64 += shp[l];
    const double target =
        uniform53(philox_block(seed, sample, (uint32_t)t)) * T64;
    // owner lane: first with lo <= target < lo + P (P > 0), else the last with mass
    int owner = -1, lastl = -1;
    {
      double lo = 0.0;
      #pragma unroll 1
      for (int l = 0; l < 64; ++l) {
        const double hi = lo + shp[l];
        if (shp[l] > 0.0) {
          lastl = l;
          if (owner < 0 && lo <= target && target < hi) owner = l;
        }
        lo = hi;
      }
    }
    if (owner < 0) owner = lastl;
    int ch = -1;
    double Cc = 0.0, Cn = 0.0;
    if (owner >= 0) {
      double own_lo = 0.0;
      #pragma unroll 1
      for (int l = 0; l < owner; ++l) own_lo += shp[l];
      const double own_hi = own_lo + shp[owner];
      const int c0 = owner * q, cn = max(0, min(q, nch - c0));
      int lastc = -1;
      {
        double Q = 0.0;
        #pragma unroll 1
        for (int j = 0; j < cn; ++j) {
          const double v = cs[c0 + j];
          Q += v;
          const double C = (j == cn - 1) ? own_hi : own_lo + Q;
          if (v > 0.0) {
            lastc = j;
            if (ch < 0 && C > target) ch = j;
          }
        }
      }
      if (ch < 0) ch = lastc;  // rounding at the owner's end
      if (ch >= 0) {  // the chosen chunk's bounds, the same additions again
        double Q = 0.0;
        #pragma unroll 1
        for (int j = 0; j < ch; ++j) Q += cs[c0 + j];
        Cc = ch == 0 ? own_lo : own_lo + Q;
        Cn = ch == cn - 1 ? own_hi : own_lo + (Q + cs[c0 + ch]);
        ch += c0;
      }
    }
    sc[0] = ch;
    sv[0] = Cc;
    sv[1] = Cn;
    sv[2] = target;
  }
  wave_sync();
  const int ch = sc[0];
  if (ch >= 0)
    #pragma unroll 1
    for (int j = lane; j < RCHUNK; j += 64) wl[j] = wr[(size_t)ch * RCHUNK + j];
  wave_sync();
  if (lane == 0) {
    int site = -1;
    if (ch >= 0) {
      const double Cc = sv[0], Cn = sv[1], target = sv[2];
      double Pp = 0.0;
      int xx = -1, last = -1;
      #pragma unroll 1
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
    sc[1] = site;
  }
  wave_sync();
  return sc[1];
}

// Lists local sample s for a replay once (div[s] set); the row within the
// call's chunk and the Philox sample index go to slot rep_ctl[1]++.
__device__ inline void list_replay(int32_t* div, int32_t* rep_ctl, int32_t* rep_row,
                                   uint64_t* rep_sid, int row0, const uint64_t* sid,
                                   uint64_t first, int s) {
  if (atomicOr(&div[s], 1) == 0) {
    const int i = atomicAdd(&rep_ctl[1], 1);
    rep_row[i] = row0 + s;
    rep_sid[i] = sample_index(sid, first, s);
  }
}

// Dense float64 Gamma of sample s's current step into row `row` of dst
// ([rows][Np]): e_{m_t} - sum_{i<t} beta_i e_{m_i} from the step's beta.
__device__ inline void dense_gamma(const DArgs& a, int s, int lane, void* dst, int row) {
  const int32_t* pm = a.perm + (size_t)s * a.N;
  const int32_t* cm = a.cmap ? a.cmap + (size_t)s * a.N : nullptr;
  if (a.cplx) {
    double2* g = reinterpret_cast<double2*>(dst) + (size_t)row * a.Np;
    const double2* bv = reinterpret_cast<const double2*>(a.beta) + (size_t)s * a.N;
    for (int k = lane; k < a.Np; k += 64) g[k] = make_double2(0.0, 0.0);
    __threadfence_block();  // the zeros land before any lane's scatter
    wave_sync();
    for (int i = lane; i <= a.t; i += 64)
      g[cm ? cm[pm[i]] : pm[i]] = (i == a.t) ? make_double2(1.0, 0.0) : make_double2(-bv[i].x, -bv[i].y);
  } else {
    double* g = reinterpret_cast<double*>(dst) + (size_t)row * a.Np;
    const double* bv = reinterpret_cast<const double*>(a.beta) + (size_t)s * a.N;
    for (int k = lane; k < a.Np; k += 64) g[k] = 0.0;
    __threadfence_block();  // the zeros land before any lane's scatter
    wave_sync();
    for (int i = lane; i <= a.t; i += 64) g[cm ? cm[pm[i]] : pm[i]] = (i == a.t) ? 1.0 : -bv[i];
  }
}

// Draw of sample s by one wavefront (lane); shp[64] is this wavefront's LDS
// scratch.  DEFER: flagged draws are recorded (a.rec_meta), else queued for
// the per-step redraw.
template <bool DEFER>
__device__ inline void draw_one(const DArgs& a, int s, int lane, double* shp) {
  const int nblk = a.L_pad / 32;
  int32_t* xrow = a.xs + (size_t)s * a.N;
  uint32_t* oc = a.occ + (size_t)s * nblk;
  if (lane == 0 && a.fslot) a.fslot[s] = -1;  // set below when the draw is flagged
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
  if constexpr (DEFER) {
    // deferred: keep the float32 site and record the draw for the float64
    // check at the end of the call (a sample whose record does not fit is
    // listed for a replay at once)
    int r = 0;
    if (lane == 0) {
      r = atomicAdd(&a.rec_ctl[0], 1);
      atomicAdd(&a.counters[0], 1ull);
    }
    r = __shfl(r, 0, 64);
    if (r < a.rec_cap) {
      uint32_t* ro = a.rec_occ + (size_t)r * nblk;
      for (int i = lane; i < nblk; i += 64) ro[i] = oc[i];  // before this draw's bit
      dense_gamma(a, s, lane, a.rec_g, r);
      if (lane == 0) {
        int32_t* m = a.rec_meta + 4 * (size_t)r;
        m[0] = s;
        m[1] = a.t;
        m[2] = site;
        m[3] = 0;
      }
    } else if (lane == 0) {
      list_replay(a.div, a.rec_ctl, a.rep_row, a.rep_sid, a.row0, a.sid, a.first, s);
    }
    wave_sync();
    if (lane == 0) {
      xrow[a.t] = site;
      atomicOr(&oc[site >> 5], 1u << (site & 31));
    }
  } else {
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
    dense_gamma(a, s, lane, a.g64, slot);
  }
}

}  // namespace ffsk
