// Batched all-site weight evaluation (the "2Lk inner products" of the cost
// count after Eq. (3)) for S samples sharing one U, as one contraction per
// step on the FP32 matrix cores:
//
//   V = U . Gamma      (L_pad x K) . (K x S),  w(x, s) = |V(x, s)|^2
//
// Real U: K = Np and Gamma[s] is the dense N-vector of step t (1 at m_t,
// -beta at m_<t).  Complex U (the bilinear u^T h of Eq. (3)) takes Gauss's
// three-multiplication form of a complex product: three real products over
// K = Np,
//   P1 = Ur Gr,  P2 = Ui Gi,  P3 = (Ur + Ui)(Gr + Gi),
// give V_re = P1 - P2 and V_im = (P3 - P1) - P2; w = V_re^2 + V_im^2.  That
// is 6 L Np S flops per launch where the real embedding [Ur | Ui] against
// [Gr ; -Gi] and [Gi ; Gr] runs 8 L Np S; the sums Ur + Ui and Gr + Gi are
// rounded to float32 in registers as the operands are read.
//
// Epilogue (fused): occupied sites get weight 0; w is stored in float32
// [S][L_pad]; float64 sums of each aligned 32-site block are stored in
// [S][L_pad/32] for the inverse-CDF scan.
//
// Tiling: 256 threads (4 wavefronts), workgroup tile 128 sites x 128 GEMM
// columns, each wavefront 64 x 64 as 2 x 2 v_mfma_f32_32x32x2f32 tiles
// (complex: 64 sites x 32 samples as 2 x 3 tiles, one per product);
// K in chunks of 32 through double-buffered LDS (one barrier per chunk, the
// next chunk's global loads in flight during the current chunk's MFMAs).
// Every output element is accumulated over K in the same fixed order
// whatever its tile, so results do not depend on the batch size or on which
// tile a sample falls in.
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

// LDS row padding of the B tile of a K chunk of kc.  Staging writes B
// transposed, one float per store: in a half-wavefront, lane (j, q) writes row
// 4q + c, column j, with kc/4 k-quads q and 32/(kc/4) samples j.  For kc = 32
// (4 samples x 8 quads) a row stride of TN + 1 floats (TN a multiple of 32)
// puts those 32 addresses in 32 different banks (a stride of TN + 4 put them
// in 8: a 4-way conflict on every staging store); for kc = 16 (8 samples x 4
// quads) a stride of TN + 2 does.  The MFMA operand reads (32 consecutive
// floats of one row per half-wavefront) are conflict-free with any stride.
__host__ __device__ constexpr int bpad(int kc) { return kc == 16 ? 2 : 1; }

// Up to four staging registers without an array: an array captured by the
// staging lambdas is kept in private (scratch) memory, which makes every
// prefetched load complete before the MFMAs can start.  With a constant
// index (all loops below are unrolled) get/put fold to a plain register.
struct Stage4 {
  float4 v0, v1, v2, v3;
};
__device__ __forceinline__ float4 get(const Stage4& s, int h) {
  switch (h) {
    case 0: return s.v0;
    case 1: return s.v1;
    case 2: return s.v2;
    default: return s.v3;
  }
}
__device__ __forceinline__ void put(Stage4& s, int h, float4 x) {
  switch (h) {
    case 0: s.v0 = x; break;
    case 1: s.v1 = x; break;
    case 2: s.v2 = x; break;
    default: s.v3 = x;
  }
}

// One TM-site x TN-column tile (bx, by) of the float32 contraction.  Four
// wavefronts as 2 x 2, each (TM/2) x (TN/2) as 32 x 32 accumulator tiles; K
// staged through double-buffered LDS in chunks of KC.  Whatever the tile
// shape and chunk, every output accumulates over K in the same order (two k
// per MFMA, ascending), so the variants give bit-identical results and
// differ only in speed: KC = 16 halves the LDS of a tile, so twice as many
// workgroups share a CU and hide each other's loads, barriers and epilogues.
template <bool CPLX, int TM, int TN, int KC>
__device__ inline void weights_tile(const WArgs& g, int bx, int by) {
  static_assert(!CPLX || TN == 128, "complex tiles hold [Gr | Gi] pairs of 32 columns");
  constexpr int AW = CPLX ? 2 * TM : TM;       // A tile row: [Ur | Ui] for complex
  static_assert(KC == 16 || KC == 32, "K chunk");
  constexpr int RT = TM / 64, CT = TN / 64;   // accumulator tiles per wavefront
  constexpr int TPR = TM / 4;                 // A staging threads per k row
  constexpr int RPP = 256 / TPR;              // k rows per A staging pass
  constexpr int PA = KC / RPP;                // A float4 per thread
  constexpr int KQ = KC / 4;                  // k-quads per chunk
  constexpr int SPP = 256 / KQ;               // samples per B staging pass
  constexpr int PB = CPLX ? 2 * (64 / SPP) : TN / SPP;  // B float4 per thread
  constexpr int BP = bpad(KC);
  __shared__ float As[2][KC][AW];
  __shared__ float Bs[2][KC][TN + BP];
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int wm = (wave & 1) * (TM / 2);   // wave's site offset in the tile
  const int wn = (wave >> 1) * (TN / 2);  // wave's GEMM-column offset in the tile
  const int site0 = bx * TM;
  // GEMM columns of the tile: real -> samples smp0..smp0+TN-1; complex ->
  // samples smp0..smp0+63 laid out per wavefront as [Gr(32) | Gi(same 32)].
  const int K = g.N;
  const int smp0 = by * (CPLX ? TN / 2 : TN);

  // staging thread map: A rows kk = a_kk + RPP*h, columns a_col..a_col+3;
  // B samples j = b_j + SPP*h, k-quads kq = b_kq
  const int a_kk = tid / TPR, a_col = (tid % TPR) * 4;
  const int b_j = tid / KQ, b_kq = tid % KQ;
  static_assert(PA >= 1 && PA <= 4 && PB >= 1 && PB <= 4, "staging holds four float4");
  Stage4 ra, ri, rb;  // ri: the Ui rows of a complex chunk
  const size_t a_off = (size_t)a_kk * g.L_pad + site0 + a_col;
  auto load_chunk = [&](int kc) {
    const float* pa = g.ut + (size_t)kc * g.L_pad + a_off;
#pragma unroll
    for (int h = 0; h < PA; ++h)
      put(ra, h, *reinterpret_cast<const float4*>(pa + (size_t)h * RPP * g.L_pad));
    if (CPLX) {
      const float* pi = pa + (size_t)g.N * g.L_pad;
#pragma unroll
      for (int h = 0; h < PA; ++h)
        put(ri, h, *reinterpret_cast<const float4*>(pi + (size_t)h * RPP * g.L_pad));
    }
    if (!CPLX) {
      const float* pb = g.gam + (size_t)(smp0 + b_j) * g.Kg + kc + 4 * b_kq;
#pragma unroll
      for (int h = 0; h < PB; ++h)
        put(rb, h, *reinterpret_cast<const float4*>(pb + (size_t)h * SPP * g.Kg));
    } else {  // per sample: Gr and Gi of the chunk's k
      const int k = kc + 4 * b_kq;
#pragma unroll
      for (int h = 0; h < PB / 2; ++h) {
        const float* r = g.gam + (size_t)(smp0 + b_j + SPP * h) * g.Kg;
        put(rb, 2 * h, *reinterpret_cast<const float4*>(r + k));
        put(rb, 2 * h + 1, *reinterpret_cast<const float4*>(r + g.N + k));
      }
    }
  };
  auto put_b = [&](int buf, int col, float4 v) {
    Bs[buf][4 * b_kq + 0][col] = v.x;
    Bs[buf][4 * b_kq + 1][col] = v.y;
    Bs[buf][4 * b_kq + 2][col] = v.z;
    Bs[buf][4 * b_kq + 3][col] = v.w;
  };
  auto store_chunk = [&](int buf) {
#pragma unroll
    for (int h = 0; h < PA; ++h)
      *reinterpret_cast<float4*>(&As[buf][a_kk + RPP * h][a_col]) = get(ra, h);
    if (CPLX) {
#pragma unroll
      for (int h = 0; h < PA; ++h)
        *reinterpret_cast<float4*>(&As[buf][a_kk + RPP * h][TM + a_col]) = get(ri, h);
    }
    if (!CPLX) {
#pragma unroll
      for (int h = 0; h < PB; ++h) put_b(buf, b_j + SPP * h, get(rb, h));
    } else {  // sample j < 32: Gr column j, Gi column j + 32 (wave block 0);
              // sample j >= 32: columns 64 + (j - 32) and 96 + (j - 32) (block 1)
#pragma unroll
      for (int h = 0; h < PB / 2; ++h) {
        const int j = b_j + SPP * h;
        const int c0 = (j >= 32 ? 64 : 0) + (j & 31);
        put_b(buf, c0, get(rb, 2 * h));
        put_b(buf, c0 + 32, get(rb, 2 * h + 1));
      }
    }
  };

  // real: CT sample tiles per site tile; complex: the products P1, P2, P3
  constexpr int NA = CPLX ? 3 : CT;
  floatx16 acc[RT][NA];
#pragma unroll
  for (int i = 0; i < RT; ++i)
#pragma unroll
    for (int j = 0; j < NA; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;

  load_chunk(0);
  store_chunk(0);
  __syncthreads();
  int buf = 0;
  const int li = lane & 31, kh = lane >> 5;
  for (int kc = 0; kc < K; kc += KC) {
    const bool more = kc + KC < K;
    if (more) load_chunk(kc + KC);
#pragma unroll
    for (int kk = 0; kk < KC; kk += 2) {
      const int kr = kk + kh;
      float a[RT], b[CT];
#pragma unroll
      for (int i = 0; i < RT; ++i) a[i] = As[buf][kr][wm + 32 * i + li];
#pragma unroll
      for (int j = 0; j < CT; ++j) b[j] = Bs[buf][kr][wn + 32 * j + li];
      if constexpr (CPLX) {  // b = {Gr, Gi} of the wavefront's 32 samples
        const float bs = b[0] + b[1];
#pragma unroll
        for (int i = 0; i < RT; ++i) {
          const float ai = As[buf][kr][TM + wm + 32 * i + li];
          const float as = a[i] + ai;
          acc[i][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i], b[0], acc[i][0], 0, 0, 0);
          acc[i][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(ai, b[1], acc[i][1], 0, 0, 0);
          acc[i][2] = __builtin_amdgcn_mfma_f32_32x32x2f32(as, bs, acc[i][2], 0, 0, 0);
        }
      } else {
#pragma unroll
        for (int i = 0; i < RT; ++i)
#pragma unroll
          for (int j = 0; j < CT; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i], b[j], acc[i][j], 0, 0, 0);
      }
    }
    if (more) {
      store_chunk(buf ^ 1);
      __syncthreads();
      buf ^= 1;
    }
  }

  // ---- epilogue -------------------------------------------------------------
  const int nblk = g.L_pad / 32;
  if constexpr (!CPLX && TM == 64 && TN == 64) {
    // one 32 x 32 tile per wavefront: its weights staged in LDS (the tile's
    // operand buffers, free once every wavefront is past its last read) and
    // streamed out as whole sample lines
    __syncthreads();
    float* st = wave < 2 ? &As[0][0][0] + wave * 1024 : &Bs[0][0][0] + (wave - 2) * 1024;
    wk::epilogue_lines(g, nblk, site0 + wm, smp0 + wn, li, kh, acc[0][0], st);
    return;
  }
#pragma unroll
  for (int i = 0; i < RT; ++i) {
    if constexpr (CPLX) {
      floatx16 re, im;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        re[r] = acc[i][0][r] - acc[i][1][r];
        im[r] = (acc[i][2][r] - acc[i][0][r]) - acc[i][1][r];
      }
      epilogue<true>(g, nblk, site0 + wm + 32 * i, smp0 + (wn >> 1) + li, kh, re, im);
    } else {
#pragma unroll
      for (int j = 0; j < CT; ++j)
        epilogue<false>(g, nblk, site0 + wm + 32 * i, smp0 + wn + 32 * j + li, kh, acc[i][j],
                        acc[i][j]);
    }
  }
}

// OCC: wavefronts per SIMD the register budget is cut for (LDS allows
// 160 KB / the tile's LDS workgroups per CU).
template <bool CPLX, int TM, int TN, int KC, int OCC>
__global__ __launch_bounds__(256, OCC) void weights_kernel(WArgs g) {
  stamp_start(g);
  weights_tile<CPLX, TM, TN, KC>(g, blockIdx.x, blockIdx.y);
  stamp_end(g);
}

// Grouped contraction: the tiles of every active instance of a list, each
// block taking items blockIdx.x, blockIdx.x + gridDim.x, ...  (K chunk 32,
// complex 16: the three complex accumulators and a 32-wide chunk's staging
// do not fit two wavefronts per SIMD).
template <bool CPLX, int TM, int TN>
__global__ __launch_bounds__(256, 2) void weights_group_kernel(const GInst* inst, GList l) {
  for (int item = blockIdx.x; item < l.total; item += gridDim.x) {
    const int k = glist_find(l, item);
    const GInst* I = inst + l.ids[k];
    const int t = I->t;
    if (t < 0 || t >= I->n_keep) continue;
    const WArgs g = I->wa;
    const int local = item - l.pre[k];
    const int gx = g.L_pad / TM;
    weights_tile<CPLX, TM, TN, CPLX ? 16 : 32>(g, local % gx, local / gx);
    __syncthreads();  // LDS of this tile is free before the next
  }
}

}  // namespace

void launch_weights(const Dims& d, const Work& w, const void* ubulk_t,
                    const void* ubf, int S, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1,
                    unsigned long long* stamp) {
  WArgs g = make_wargs(d, w, ubulk_t);
  g.stamp = stamp;
  const int s_round = (S + SAMPLE_PAD - 1) / SAMPLE_PAD * SAMPLE_PAD;
  if (d.bf16) {
    launch_weights_bf16(d, g, ubf, s_round, st, ev0, ev1);
    return;
  }
  launch_weights_variant(d, g, s_round, tile_choice(d, s_round), st, ev0, ev1);
}

int weights_group_items(const Dims& d, int S, int v) {
  const int s_round = (S + SAMPLE_PAD - 1) / SAMPLE_PAD * SAMPLE_PAD;
  return (d.L_pad / kTiles[v].sites) * (s_round / (d.cplx ? kTiles[v].cols / 2 : kTiles[v].cols));
}

// ---- tile variants of the float32 contraction ---------------------------
// {sites, GEMM columns, K chunk, the variant of the same tile with a 32-wide
// chunk (what grouped launches run: identical results)}
const TileShape kTiles[kNumTilesDecl] = {{128, 128, 32, 0}, {64, 128, 32, 1}, {128, 64, 32, 2},
                                         {64, 64, 32, 3},   {128, 128, 16, 0}, {64, 128, 16, 1},
                                         {128, 64, 16, 2},  {64, 64, 16, 3}};

bool tile_allowed(const Dims& d, int v) { return !d.cplx || kTiles[v].cols == 128; }

void launch_weights_variant(const Dims& d, const WArgs& g, int s_round, int v,
                            hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  const int tm = kTiles[v].sites, tn = kTiles[v].cols;
  const dim3 grid(d.L_pad / tm, s_round / (d.cplx ? tn / 2 : tn));
  if (d.cplx) {
    switch (v) {
      case 1: launch256(weights_kernel<true, 64, 128, 32, 3>, grid, st, ev0, ev1, g); break;
      case 4: launch256(weights_kernel<true, 128, 128, 16, 3>, grid, st, ev0, ev1, g); break;
      case 5: launch256(weights_kernel<true, 64, 128, 16, 4>, grid, st, ev0, ev1, g); break;
      default: launch256(weights_kernel<true, 128, 128, 32, 2>, grid, st, ev0, ev1, g);
    }
    return;
  }
  switch (v) {
    case 1: launch256(weights_kernel<false, 64, 128, 32, 3>, grid, st, ev0, ev1, g); break;
    case 2: launch256(weights_kernel<false, 128, 64, 32, 3>, grid, st, ev0, ev1, g); break;
    case 3: launch256(weights_kernel<false, 64, 64, 32, 4>, grid, st, ev0, ev1, g); break;
    case 4: launch256(weights_kernel<false, 128, 128, 16, 4>, grid, st, ev0, ev1, g); break;
    case 5: launch256(weights_kernel<false, 64, 128, 16, 6>, grid, st, ev0, ev1, g); break;
    case 6: launch256(weights_kernel<false, 128, 64, 16, 6>, grid, st, ev0, ev1, g); break;
    case 7: launch256(weights_kernel<false, 64, 64, 16, 8>, grid, st, ev0, ev1, g); break;
    default: launch256(weights_kernel<false, 128, 128, 32, 2>, grid, st, ev0, ev1, g);
  }
}

WArgs make_wargs(const Dims& d, const Work& w, const void* ubulk_t) {
  WArgs g;
  g.ut = static_cast<const float*>(ubulk_t);
  g.gam = static_cast<const float*>(w.gam);
  g.occ = w.occ;
  g.wh = static_cast<float*>(w.wh);
  g.bsum = w.bsum;
  g.stamp = nullptr;
  g.L_pad = d.L_pad;
  g.N = d.Np;
  g.Kg = d.Kg;
  g.S_pad = w.S_pad;
  return g;
}

void launch_weights_group(const GInst* inst, const GList& l, bool cplx, int v,
                          hipStream_t st) {
  if (l.total == 0) return;
  const int grid = l.total < 2048 ? l.total : 2048;
  if (cplx) {
    if (v == 1)
      hipLaunchKernelGGL((weights_group_kernel<true, 64, 128>), dim3(grid), dim3(256), 0, st, inst, l);
    else
      hipLaunchKernelGGL((weights_group_kernel<true, 128, 128>), dim3(grid), dim3(256), 0, st, inst, l);
    return;
  }
  switch (v) {
    case 1:
      hipLaunchKernelGGL((weights_group_kernel<false, 64, 128>), dim3(grid), dim3(256), 0, st, inst, l);
      break;
    case 2:
      hipLaunchKernelGGL((weights_group_kernel<false, 128, 64>), dim3(grid), dim3(256), 0, st, inst, l);
      break;
    case 3:
      hipLaunchKernelGGL((weights_group_kernel<false, 64, 64>), dim3(grid), dim3(256), 0, st, inst, l);
      break;
    default:
      hipLaunchKernelGGL((weights_group_kernel<false, 128, 128>), dim3(grid), dim3(256), 0, st, inst, l);
  }
}

}  // namespace ffsk
