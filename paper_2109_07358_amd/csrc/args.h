// Per-launch argument blocks of the batched kernels, and the device table of
// the grouped (multi-instance) executor that holds one block of each per
// instance.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ffsk {

// All-site weight contraction (k_weights.hip).
struct WArgs {
  const float* ut;       // [K][L_pad] k-major bulk U (complex: Ur rows, then Ui)
  const float* gam;      // [S_pad][Kg] (split-BF16: [S_pad][Kg/16][16 heads | 16 tails] bfloat16)
  const uint32_t* occ;   // [S_pad][L_pad/32]
  float* wh;             // [S_pad][L_pad]
  double* bsum;          // [S_pad][L_pad/32]
  // measurement hook, nullable: [0] earliest workgroup start, [1] latest
  // workgroup end of the launch, in steady-clock ticks (min / max updates)
  unsigned long long* stamp;
  int L_pad, N, Kg, S_pad;
};

// Inverse-CDF draw with guard (k_draw.hip).
struct DArgs {
  const double* bsum;  // [S_pad][nblk]
  const float* wh;     // [S_pad][L_pad]
  int32_t* xs;         // [S_pad][N]
  uint32_t* occ;       // [S_pad][nblk]
  int32_t* ctl;        // [0] flag count, [1] status
  int32_t* flag_list;
  unsigned long long* counters;
  const int32_t* forced;
  const int32_t* perm;  // [S_pad][N]
  const void* beta;     // [S_pad][N] float64 / complex128
  void* g64;            // [S_pad][Np] dense float64 Gamma per flag slot
  const int32_t* cmap;  // [S_pad][N] per-sample columns of U, or null
  const uint64_t* sid;  // [S] Philox sample index per sample, or null (first + s)
  int32_t* fslot;       // [S_pad] redraw slot of the sample's draw, -1 if not flagged
                        // (null when flagged draws are recorded instead)
  // Deferred resolution (rec_meta non-null): a flagged draw keeps its
  // float32 site and is recorded for one float64 check at the end of the
  // call; a sample whose record does not fit is listed for a replay at once.
  int32_t* rec_meta;    // [rec_cap][4] sample, step, float32 site, 0
  void* rec_g;          // [rec_cap][Np] dense float64 Gamma of the draw
  uint32_t* rec_occ;    // [rec_cap][L_pad/32] occupancy before the draw
  int32_t* rec_ctl;     // [0] records taken, [1] samples listed for replay
  int32_t* div;         // [S_pad] 1 once the sample is listed
  int32_t* rep_row;     // [S_pad] listed samples' rows in the call's chunk
  uint64_t* rep_sid;    // [S_pad] their Philox sample indices
  int rec_cap, row0;    // row0: row of local sample 0 in the chunk
  int S, L_pad, N, Np, t, n_forced, cplx;
  // guard threshold of a draw: max(delta * T, coef * sqrt(sum_b B_b^2)),
  // B_b the float64 32-site block sums (coef = 0: fixed relative margin)
  double delta, coef;
  uint64_t seed, first;
};

// Float64 redraw of flagged draws (k_draw.hip).
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
  double* cs;          // [S_pad][nch]   their 64-site chunk sums
  void* g64;           // [S_pad][Np]    their dense float64 Gamma
  const uint64_t* sid; // [S] Philox sample index per sample, or null (first + s)
  // Records of a deferred call (occ_rec non-null): slots rec_base ..
  // rec_base + rec_span - 1 of the records taken (ctl[0], at most rec_cap),
  // occ_rec / g64 already offset to rec_base; slot f's occupancy is
  // occ_rec[f], and flag_list is not read.
  const uint32_t* occ_rec;
  int rec_base, rec_span, rec_cap;
  int L_pad, N, Np, K, t;  // N particles (xs stride), K columns of U
  uint64_t seed, first;
};

// End-of-call float64 check of the recorded draws (k_draw.hip): record
// rec_base + f against the float64 weights wr[f] / chunk sums cs[f].
struct VArgs {
  const int32_t* rec_meta;
  const int32_t* rec_ctl;
  const double* wr;
  const double* cs;
  int32_t* ctl;                 // [1] device status
  unsigned long long* counters; // [1] changed
  int32_t* div;
  int32_t* rep_row;
  uint64_t* rep_sid;
  int32_t* rep_ctl;             // [1] samples listed
  const uint64_t* sid;
  int L_pad, rec_base, rec_span, rec_cap, row0;
  uint64_t seed, first;
};

// Float64 factor update / solve, one wavefront per sample (k_batched.hip).
// A launch that absorbs step t first finishes the float64 redraw of the
// samples whose draw at t was flagged (fslot, wr, cs from the redraw product).
struct FArgs {
  const void* u64;
  void* F;
  int32_t* perm;
  int32_t* xs;
  const int32_t* fslot;        // [S_pad] redraw slot or -1
  const double* wr;            // [slots][L_pad] float64 weights of flagged draws
  const double* cs;            // [slots][L_pad/64] their 64-site chunk sums
  uint32_t* occ;               // [S_pad][L_pad/32]
  unsigned long long* counters;
  void* beta;
  double* logdet;
  int32_t* ctl;
  float* gam;
  // split-BF16 plans: Gamma written as bfloat16 heads and tails (the
  // contraction's operands) instead of float32, in the same bytes: per
  // sample [Kg/16][16 heads | 16 tails]; else null
  uint16_t* gsplit;
  const int32_t* cmap;  // [S_pad][N] per-sample columns of U, or null
  const uint64_t* sid;  // [S] Philox sample index per sample, or null (first + s)
  int N, Np, Kg, ldu, L_pad, t_upd, t_solve, n_steps;
  uint64_t seed, first;
};

// One instance of the grouped executor.  `t` is the step its next tick
// performs; it lives in device memory and is advanced on the device at the
// end of every tick, so a captured sequence of ticks can be replayed.
struct GInst {
  WArgs wa;
  const uint16_t* uh;  // split-BF16 plans: bfloat16 heads and tails of U
  const uint16_t* ul;  // ([Kg/32][L_pad][32] each), else null
  DArgs da;
  RArgs ra;
  FArgs fa;
  int t, n_keep, S, cplx;
};

// Work items of one grouped launch: instances ids[0..n) with item counts
// given by the prefix pre[0..n] (pre[0] = 0, pre[n] = total).
struct GList {
  const int* ids;
  const int* pre;
  int n, total;
};

// Philox sample index of local sample s of a launch.
__device__ inline uint64_t sample_index(const uint64_t* sid, uint64_t first, int s) {
  return sid ? sid[s] : first + (uint64_t)s;
}

// Instance of item `item` (pre non-decreasing): largest k with pre[k] <= item.
__device__ inline int glist_find(const GList& l, int item) {
  int lo = 0, hi = l.n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (l.pre[mid] <= item)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

}  // namespace ffsk
