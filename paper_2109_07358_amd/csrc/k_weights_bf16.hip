// Split-BF16 all-site weight contraction: the same product and fused
// epilogue as the float32 contraction (k_weights.hip), on the bfloat16
// matrix cores.
#include <hip/hip_ext.h>

#include "args.h"
#include "ffs_internal.h"
#include "weights_common.h"

namespace ffsk {

using wk::epilogue;
using wk::launch256;
using wk::stamp_end;
using wk::stamp_start;

namespace {

constexpr int MT = 128;  // sites per workgroup tile
constexpr int NT = 128;  // GEMM columns per workgroup tile

// U = Uh + Ul and Gamma = Gh + Gl with bfloat16 heads and tails (the tail is
// the bfloat16 rounding of what the head leaves), and V = Uh Gh + Uh Gl + Ul Gh
// on v_mfma_f32_32x32x16_bf16 with float32 accumulation, in that fixed order
// per K step; Ul Gl lies below the float32 accumulation error.  Same tile
// (128 sites x 128 GEMM columns, 4 wavefronts of 64 x 64) and epilogue as the
// float32 kernel.  U's heads and tails are stored chunk-major,
// [Kg/32][L_pad][32], so one 128-site x 32-k tile is 8 KB of contiguous
// memory.  Gamma arrives split too: the factor update writes, in place of the
// float32 Gamma, per sample and per 16-wide block of k, 16 bfloat16 heads
// and then their 16 tails, so a column's block is one 64-byte run.  K goes in
// chunks of 16 (one MFMA k-step) through double-buffered LDS holding head and
// tail tiles: 32 KB per workgroup, four workgroups per CU.  (Chunks of 32
// give the same MFMA sequence, hence the same bits, with half the
// workgroups per CU, and measured 3-4% slower.)

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
constexpr int BK = 32;   // K chunk of U's global layout
constexpr int BKS = 16;  // K chunk staged through LDS

// bfloat16 offset of 16-byte half qt (0..1) of LDS row r (32 B per row).
// Measured on gfx950 (SQ_LDS_BANK_CONFLICT): a 16-byte LDS read serves 16
// consecutive lanes at a time and conflicts where two of them meet modulo
// 256 B; a 16-byte write serves 8 lanes at a time, conflicting modulo 128 B.
// The halves are XOR-swizzled by (r / 8) % 2, so an MFMA operand read (16
// lanes, one half of 16 consecutive rows) covers 256 B once, and an A
// staging store (8 lanes, 4 rows x 2 halves) 128 B once.  The tail tile of B
// takes row r ^ 2 for column r: a B staging store's 8 lanes write 2
// columns' heads and the same 2 columns' tails, the two tiles lie 8 KB
// apart, and the shift puts the tails in the other half of the 128 B.
__device__ __forceinline__ int swq16(int r, int qt) { return r * 16 + 8 * (qt ^ ((r >> 3) & 1)); }

struct WArgsB {
  WArgs o;             // Gamma, occupancy and outputs as in the float32 kernel
  const uint16_t* uh;  // [Kg/32][L_pad][32] bfloat16 heads of U
  const uint16_t* ul;  // tails, same layout
};

// One MT x NT tile (bx, by) of the split-BF16 contraction.  Each
// accumulator sees, per 16 k in ascending order, head x head, head x tail,
// tail x head.
template <bool CPLX>
__device__ inline void weights_bf16_tile(const WArgsB& a, int bx, int by) {
  static_assert(MT * 2 == 256 && NT * 4 == 512, "staging: one A piece, two B pieces per thread");
  const WArgs& g = a.o;
  const uint16_t* gs = reinterpret_cast<const uint16_t*>(g.gam);
  __shared__ __align__(16) uint16_t Ah[2][MT * BKS];
  __shared__ __align__(16) uint16_t Al[2][MT * BKS];
  __shared__ __align__(16) uint16_t Bs[2][2][NT * BKS];  // [buffer][heads, tails]
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int wm = (wave & 1) * 64;
  const int wn = (wave >> 1) * 64;
  const int site0 = bx * MT;
  const int K = CPLX ? 2 * g.N : g.N;
  const int smp0 = by * (CPLX ? NT / 2 : NT);

  // A staging: MT rows x 2 halves, one 16-byte piece per thread; U's
  // 32-wide global chunks hold a 16-wide chunk in the first or second half
  // of each site's 64 bytes.  B staging: NT columns x 4 pieces (heads of k
  // 0..7, 8..15, then tails), two per thread, consecutive lanes on a
  // column's consecutive pieces.  Complex columns hold [re | im] pairs per
  // wavefront block (column j + 32 part, + 32 for samples 32..63) of
  // B_re = [Gr; -Gi], B_im = [Gi; Gr] over K = 2 Np; the negated block flips
  // sign bits (bf16 rounding is symmetric, so this equals splitting the
  // negated value).
  uint4 rah, ral, rb0, rb1;
  auto ld_b = [&](int c, int kc) {
    const int col = c >> 2, sub = c & 3;
    int j, k0;
    bool neg = false;
    if (!CPLX) {
      j = col;
      k0 = kc;
    } else {
      const int wi = col & 63, part = wi >> 5;
      j = (col >> 6) * 32 + (wi & 31);
      const bool top = kc < g.N;
      k0 = part ? (top ? kc + g.N : kc - g.N) : kc;
      neg = !part && !top;
    }
    // block k0 / 16 of the sample's row starts at bfloat16 offset 2 k0
    uint4 v = *reinterpret_cast<const uint4*>(gs + (size_t)(smp0 + j) * 2 * g.Kg + 2 * k0 + 8 * sub);
    if (neg) {
      v.x ^= 0x80008000u;
      v.y ^= 0x80008000u;
      v.z ^= 0x80008000u;
      v.w ^= 0x80008000u;
    }
    return v;
  };
  auto st_b = [&](int buf, int c, uint4 v) {
    const int col = c >> 2, sub = c & 3;
    const int tail = sub >> 1;
    *reinterpret_cast<uint4*>(&Bs[buf][tail][swq16(col ^ (2 * tail), sub & 1)]) = v;
  };
  auto load_chunk = [&](int kc) {
    const size_t off = ((size_t)(kc / BK) * g.L_pad + site0 + (tid >> 1)) * BK + (kc % BK) + 8 * (tid & 1);
    rah = *reinterpret_cast<const uint4*>(a.uh + off);
    ral = *reinterpret_cast<const uint4*>(a.ul + off);
    rb0 = ld_b(tid, kc);
    rb1 = ld_b(tid + 256, kc);
  };
  auto store_chunk = [&](int buf) {
    *reinterpret_cast<uint4*>(&Ah[buf][swq16(tid >> 1, tid & 1)]) = rah;
    *reinterpret_cast<uint4*>(&Al[buf][swq16(tid >> 1, tid & 1)]) = ral;
    st_b(buf, tid, rb0);
    st_b(buf, tid + 256, rb1);
  };

  floatx16 acc00, acc01, acc10, acc11;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    acc00[r] = 0.0f;
    acc01[r] = 0.0f;
    acc10[r] = 0.0f;
    acc11[r] = 0.0f;
  }

  load_chunk(0);
  store_chunk(0);
  __syncthreads();
  int buf = 0;
  const int li = lane & 31, kh = lane >> 5;
  for (int kc = 0; kc < K; kc += BKS) {
    const bool more = kc + BKS < K;
    if (more) load_chunk(kc + BKS);
    {
      const bf16x8 ah0 = *reinterpret_cast<const bf16x8*>(&Ah[buf][swq16(wm + li, kh)]);
      const bf16x8 ah1 = *reinterpret_cast<const bf16x8*>(&Ah[buf][swq16(wm + 32 + li, kh)]);
      const bf16x8 al0 = *reinterpret_cast<const bf16x8*>(&Al[buf][swq16(wm + li, kh)]);
      const bf16x8 al1 = *reinterpret_cast<const bf16x8*>(&Al[buf][swq16(wm + 32 + li, kh)]);
      const bf16x8 bh0 = *reinterpret_cast<const bf16x8*>(&Bs[buf][0][swq16(wn + li, kh)]);
      const bf16x8 bh1 = *reinterpret_cast<const bf16x8*>(&Bs[buf][0][swq16(wn + 32 + li, kh)]);
      const bf16x8 bl0 = *reinterpret_cast<const bf16x8*>(&Bs[buf][1][swq16((wn + li) ^ 2, kh)]);
      const bf16x8 bl1 = *reinterpret_cast<const bf16x8*>(&Bs[buf][1][swq16((wn + 32 + li) ^ 2, kh)]);
      acc00 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah0, bh0, acc00, 0, 0, 0);
      acc01 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah0, bh1, acc01, 0, 0, 0);
      acc10 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah1, bh0, acc10, 0, 0, 0);
      acc11 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah1, bh1, acc11, 0, 0, 0);
      acc00 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah0, bl0, acc00, 0, 0, 0);
      acc01 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah0, bl1, acc01, 0, 0, 0);
      acc10 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah1, bl0, acc10, 0, 0, 0);
      acc11 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah1, bl1, acc11, 0, 0, 0);
      acc00 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al0, bh0, acc00, 0, 0, 0);
      acc01 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al0, bh1, acc01, 0, 0, 0);
      acc10 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al1, bh0, acc10, 0, 0, 0);
      acc11 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al1, bh1, acc11, 0, 0, 0);
    }
    if (more) {
      store_chunk(buf ^ 1);
      __syncthreads();
      buf ^= 1;
    }
  }

  const int nblk = g.L_pad / 32;
  if (CPLX) {
    epilogue<true>(g, nblk, site0 + wm, smp0 + (wn >> 1) + li, kh, acc00, acc01);
    epilogue<true>(g, nblk, site0 + wm + 32, smp0 + (wn >> 1) + li, kh, acc10, acc11);
  } else {
    epilogue<false>(g, nblk, site0 + wm, smp0 + wn + li, kh, acc00, acc00);
    epilogue<false>(g, nblk, site0 + wm, smp0 + wn + 32 + li, kh, acc01, acc01);
    epilogue<false>(g, nblk, site0 + wm + 32, smp0 + wn + li, kh, acc10, acc10);
    epilogue<false>(g, nblk, site0 + wm + 32, smp0 + wn + 32 + li, kh, acc11, acc11);
  }
}

template <bool CPLX>
__global__ __launch_bounds__(256, 4) void weights_bf16_kernel(WArgsB a) {
  stamp_start(a.o);
  weights_bf16_tile<CPLX>(a, blockIdx.x, blockIdx.y);
  stamp_end(a.o);
}

// Grouped split-BF16 contraction: the tiles of every active instance of a
// list, each block taking items blockIdx.x, blockIdx.x + gridDim.x, ...
template <bool CPLX>
__global__ __launch_bounds__(256, 2) void weights_bf16_group_kernel(const GInst* inst, GList l) {
  for (int item = blockIdx.x; item < l.total; item += gridDim.x) {
    const int k = glist_find(l, item);
    const GInst* I = inst + l.ids[k];
    const int t = I->t;
    if (t < 0 || t >= I->n_keep) continue;
    WArgsB b;
    b.o = I->wa;
    b.uh = I->uh;
    b.ul = I->ul;
    const int local = item - l.pre[k];
    const int gx = b.o.L_pad / MT;
    weights_bf16_tile<CPLX>(b, local % gx, local / gx);
    __syncthreads();  // LDS of this tile is free before the next
  }
}

}  // namespace

void launch_weights_bf16(const Dims& d, const WArgs& g, const void* ubf, int s_round,
                         hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  WArgsB b;
  b.o = g;
  b.uh = static_cast<const uint16_t*>(ubf);
  b.ul = b.uh + (size_t)d.Kg * d.L_pad;
  if (d.cplx)
    launch256(weights_bf16_kernel<true>, dim3(d.L_pad / MT, s_round / (NT / 2)), st, ev0, ev1, b);
  else
    launch256(weights_bf16_kernel<false>, dim3(d.L_pad / MT, s_round / NT), st, ev0, ev1, b);
}

int weights_bf16_group_items(const Dims& d, int S) {
  const int s_round = (S + SAMPLE_PAD - 1) / SAMPLE_PAD * SAMPLE_PAD;
  return (d.L_pad / MT) * (s_round / (d.cplx ? NT / 2 : NT));
}

void launch_weights_bf16_group(const GInst* inst, const GList& l, bool cplx, hipStream_t st) {
  if (l.total == 0) return;
  const int grid = l.total < 2048 ? l.total : 2048;
  if (cplx)
    hipLaunchKernelGGL(weights_bf16_group_kernel<true>, dim3(grid), dim3(256), 0, st, inst, l);
  else
    hipLaunchKernelGGL(weights_bf16_group_kernel<false>, dim3(grid), dim3(256), 0, st, inst, l);
}

}  // namespace ffsk
