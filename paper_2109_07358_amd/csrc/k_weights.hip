// Batched all-site weight evaluation (the "2Lk inner products" of the cost
// count after Eq. (3)) for S samples sharing one U, as one contraction per
// step on the FP32 matrix cores:
//
//   V = U . Gamma      (L_pad x K) . (K x S),  w(x, s) = |V(x, s)|^2
//
// Real U: K = Np and Gamma[s] is the dense N-vector of step t (1 at m_t,
// -beta at m_<t).  Complex U is embedded as a real product: A = [Ur | Ui]
// (L x 2Np) and two output columns per sample, B_re = [Gr ; -Gi] and
// B_im = [Gi ; Gr], so V_re = Ur Gr - Ui Gi and V_im = Ur Gi + Ui Gr (the
// bilinear u^T h of Eq. (3)); w = V_re^2 + V_im^2.
//
// Epilogue (fused): occupied sites get weight 0; w is stored in float32
// [S][L_pad]; float64 sums of each aligned 32-site block are stored in
// [S][L_pad/32] for the inverse-CDF scan.
//
// Tiling: 256 threads (4 wavefronts), workgroup tile 128 sites x 128 GEMM
// columns, each wavefront 64 x 64 as 2 x 2 v_mfma_f32_32x32x2f32 tiles;
// K in chunks of 32 through double-buffered LDS (one barrier per chunk, the
// next chunk's global loads in flight during the current chunk's 64 MFMAs
// per wavefront).  Every output element is accumulated over K in the same
// fixed order whatever its tile, so results do not depend on the batch size
// or on which tile a sample falls in.
#include <hip/hip_ext.h>

#include "args.h"
#include "ffs_internal.h"

namespace ffsk {

typedef float floatx16 __attribute__((ext_vector_type(16)));

namespace {

constexpr int MT = 128;  // sites per workgroup tile (split-bfloat16 kernel)
constexpr int NT = 128;  // GEMM columns per workgroup tile (split-bfloat16 kernel)
// LDS row padding of the B tile of a K chunk of kc.  Staging writes B
// transposed, one float per store: in a half-wavefront, lane (j, q) writes row
// 4q + c, column j, with kc/4 k-quads q and 32/(kc/4) samples j.  For kc = 32
// (4 samples x 8 quads) a row stride of TN + 1 floats (TN a multiple of 32)
// puts those 32 addresses in 32 different banks (a stride of TN + 4 put them
// in 8: a 4-way conflict on every staging store); for kc = 16 (8 samples x 4
// quads) a stride of TN + 2 does.  The MFMA operand reads (32 consecutive
// floats of one row per half-wavefront) are conflict-free with any stride.
__host__ __device__ constexpr int bpad(int kc) { return kc == 16 ? 2 : 1; }

// Epilogue of one 32 x 32 accumulator tile (sites sb..sb+31, one sample per
// lane column).  C layout: lane l, register r -> column l%32, row
// 8*(r/4) + 4*(l/32) + r%4.  Occupied sites get weight 0; the tile's sites
// form one aligned 32-site block whose float64 sum is stored.
template <bool CPLX>
__device__ inline void epilogue(const WArgs& g, int nblk, int sb, int smp, int kh,
                                floatx16 re, floatx16 im) {
  const int blk = sb >> 5;
  const uint32_t occw = g.occ[(size_t)smp * nblk + blk];
  float* dst = g.wh + (size_t)smp * g.L_pad + sb + 4 * kh;
  double part = 0.0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    float w4[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int r = 4 * q + c;
      const int row = 8 * q + 4 * kh + c;
      const float v = CPLX ? re[r] * re[r] + im[r] * im[r] : re[r] * re[r];
      w4[c] = ((occw >> row) & 1u) ? 0.0f : v;
      part += (double)w4[c];
    }
    *reinterpret_cast<float4*>(dst + 8 * q) = make_float4(w4[0], w4[1], w4[2], w4[3]);
  }
  const double other = __shfl_xor(part, 32, 64);
  const double tot = (kh == 0) ? part + other : other + part;
  if (kh == 0) g.bsum[(size_t)smp * nblk + blk] = tot;
}

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
  static_assert(!CPLX || TN == 128, "complex tiles hold [re | im] pairs of 32 columns");
  static_assert(KC == 16 || KC == 32, "K chunk");
  constexpr int RT = TM / 64, CT = TN / 64;   // accumulator tiles per wavefront
  constexpr int TPR = TM / 4;                 // A staging threads per k row
  constexpr int RPP = 256 / TPR;              // k rows per A staging pass
  constexpr int PA = KC / RPP;                // A float4 per thread
  constexpr int KQ = KC / 4;                  // k-quads per chunk
  constexpr int SPP = 256 / KQ;               // samples per B staging pass
  constexpr int PB = CPLX ? 2 * (64 / SPP) : TN / SPP;  // B float4 per thread
  constexpr int BP = bpad(KC);
  __shared__ float As[2][KC][TM];
  __shared__ float Bs[2][KC][TN + BP];
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int wm = (wave & 1) * (TM / 2);   // wave's site offset in the tile
  const int wn = (wave >> 1) * (TN / 2);  // wave's GEMM-column offset in the tile
  const int site0 = bx * TM;
  // GEMM columns of the tile: real -> samples smp0..smp0+TN-1; complex ->
  // samples smp0..smp0+63 laid out per wavefront as [re(32) | im(same 32)].
  const int K = CPLX ? 2 * g.N : g.N;
  const int smp0 = by * (CPLX ? TN / 2 : TN);

  // staging thread map: A rows kk = a_kk + RPP*h, columns a_col..a_col+3;
  // B samples j = b_j + SPP*h, k-quads kq = b_kq
  const int a_kk = tid / TPR, a_col = (tid % TPR) * 4;
  const int b_j = tid / KQ, b_kq = tid % KQ;
  static_assert(PA >= 1 && PA <= 4 && PB >= 1 && PB <= 4, "staging holds four float4");
  Stage4 ra, rb;
  const size_t a_off = (size_t)a_kk * g.L_pad + site0 + a_col;
  auto load_chunk = [&](int kc) {
    const float* pa = g.ut + (size_t)kc * g.L_pad + a_off;
#pragma unroll
    for (int h = 0; h < PA; ++h)
      put(ra, h, *reinterpret_cast<const float4*>(pa + (size_t)h * RPP * g.L_pad));
    if (!CPLX) {
      const float* pb = g.gam + (size_t)(smp0 + b_j) * g.Kg + kc + 4 * b_kq;
#pragma unroll
      for (int h = 0; h < PB; ++h)
        put(rb, h, *reinterpret_cast<const float4*>(pb + (size_t)h * SPP * g.Kg));
    } else {  // per sample: the re-part rows [Gr; -Gi] and im-part rows [Gi; Gr]
      const int k = kc + 4 * b_kq;
      const float sg = (kc < g.N) ? 1.0f : -1.0f;
      const int kim = (kc < g.N) ? k + g.N : k - g.N;
#pragma unroll
      for (int h = 0; h < PB / 2; ++h) {
        const float* r = g.gam + (size_t)(smp0 + b_j + SPP * h) * g.Kg;
        float4 re = *reinterpret_cast<const float4*>(r + k);
        re.x *= sg; re.y *= sg; re.z *= sg; re.w *= sg;
        put(rb, 2 * h, re);
        put(rb, 2 * h + 1, *reinterpret_cast<const float4*>(r + kim));
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
    if (!CPLX) {
#pragma unroll
      for (int h = 0; h < PB; ++h) put_b(buf, b_j + SPP * h, get(rb, h));
    } else {  // sample j < 32: re column j, im column j + 32 (wave block 0);
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

  floatx16 acc[RT][CT];
#pragma unroll
  for (int i = 0; i < RT; ++i)
#pragma unroll
    for (int j = 0; j < CT; ++j)
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
#pragma unroll
      for (int i = 0; i < RT; ++i)
#pragma unroll
        for (int j = 0; j < CT; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    if (more) {
      store_chunk(buf ^ 1);
      __syncthreads();
      buf ^= 1;
    }
  }

  // ---- epilogue -------------------------------------------------------------
  const int nblk = g.L_pad / 32;
#pragma unroll
  for (int i = 0; i < RT; ++i) {
    if (CPLX) {
      epilogue<true>(g, nblk, site0 + wm + 32 * i, smp0 + (wn >> 1) + li, kh, acc[i][0], acc[i][1]);
    } else {
#pragma unroll
      for (int j = 0; j < CT; ++j)
        epilogue<false>(g, nblk, site0 + wm + 32 * i, smp0 + wn + 32 * j + li, kh, acc[i][j],
                        acc[i][j]);
    }
  }
}

// Measurement hook: the launch's span on the device's steady clock, from the
// earliest start among the first workgroups dispatched (one per XCD and a
// few more) to the latest workgroup end -- the interval a kernel trace
// reports, without the dispatch and queue waits an event pair also holds.
__device__ inline void stamp_start(const WArgs& g) {
  if (g.stamp && threadIdx.x == 0 && blockIdx.x + blockIdx.y * gridDim.x < 64)
    atomicMin(&g.stamp[0], (unsigned long long)wall_clock64());
}
__device__ inline void stamp_end(const WArgs& g) {
  if (!g.stamp) return;
  __syncthreads();
  if (threadIdx.x == 0) atomicMax(&g.stamp[1], (unsigned long long)wall_clock64());
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
// block taking items blockIdx.x, blockIdx.x + gridDim.x, ...
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
    weights_tile<CPLX, TM, TN, 32>(g, local % gx, local / gx);
    __syncthreads();  // LDS of this tile is free before the next
  }
}

// ---- split-BF16 variant ------------------------------------------------------
// U = Uh + Ul and Gamma = Gh + Gl with bfloat16 heads and tails (the tail is
// the bfloat16 rounding of what the head leaves), and V = Uh Gh + Uh Gl + Ul Gh
// on v_mfma_f32_32x32x16_bf16 with float32 accumulation, in that fixed order
// per K step; Ul Gl lies below the float32 accumulation error.  Same tile
// (128 sites x 128 GEMM columns, 4 wavefronts of 64 x 64) and epilogue as the
// float32 kernel.  U's heads and tails are stored chunk-major,
// [Kg/32][L_pad][32], so one 128-site x 32-k tile is 8 KB of contiguous
// memory; Gamma (float32) is split while it is staged.  K in chunks of 32 (two
// MFMA k-steps) through double-buffered LDS holding head and tail tiles.

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
constexpr int BK = 32;    // K chunk
constexpr int BROW = 32;  // LDS row stride in bfloat16 units (64 B, unpadded)

// bfloat16 offset of 16-byte quarter qt (0..3) of LDS row r.  Quarters are
// XOR-swizzled by (r / 4) % 4: a half-wavefront's 16-byte MFMA operand reads
// (16 consecutive rows, one quarter) and the staging stores (4 consecutive
// rows, all quarters) then each cover 16 distinct 16-byte bank groups, so
// neither conflicts -- a padded stride can serve only one of the two.
__device__ __forceinline__ int swq(int r, int qt) { return r * BROW + 8 * (qt ^ ((r >> 2) & 3)); }

// bfloat16 bits of x, rounded to nearest even (x finite).
__device__ inline uint32_t bf16_rn(float x) {
  const uint32_t u = __float_as_uint(x);
  return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}

struct WArgsB {
  WArgs o;             // Gamma, occupancy and outputs as in the float32 kernel
  const uint16_t* uh;  // [Kg/32][L_pad][32] bfloat16 heads of U
  const uint16_t* ul;  // tails, same layout
};

// One MT x NT tile (bx, by) of the split-BF16 contraction.
template <bool CPLX>
__device__ inline void weights_bf16_tile(const WArgsB& a, int bx, int by) {
  const WArgs& g = a.o;
  __shared__ __align__(16) uint16_t Ah[2][MT * BROW];
  __shared__ __align__(16) uint16_t Al[2][MT * BROW];
  __shared__ __align__(16) uint16_t Bh[2][NT * BROW];
  __shared__ __align__(16) uint16_t Bl[2][NT * BROW];
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int wm = (wave & 1) * 64;
  const int wn = (wave >> 1) * 64;
  const int site0 = bx * MT;
  const int K = CPLX ? 2 * g.N : g.N;
  const int smp0 = by * (CPLX ? NT / 2 : NT);

  // A staging: 512 16-byte pieces per tile (4 per site), 2 per thread
  uint4 rah0, rah1, ral0, ral1;
  // B staging: 1024 float4 per tile, 4 per thread
  float4 rb0, rb1, rb2, rb3;
  auto load_chunk = [&](int kc) {
    const size_t base = ((size_t)(kc / BK) * g.L_pad + site0) * BK;
    rah0 = reinterpret_cast<const uint4*>(a.uh + base)[tid];
    rah1 = reinterpret_cast<const uint4*>(a.uh + base)[tid + 256];
    ral0 = reinterpret_cast<const uint4*>(a.ul + base)[tid];
    ral1 = reinterpret_cast<const uint4*>(a.ul + base)[tid + 256];
    float4* rb[4] = {&rb0, &rb1, &rb2, &rb3};
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const int c = tid + 256 * h;
      if (!CPLX) {
        const int j = c >> 3, q = c & 7;
        *rb[h] = *reinterpret_cast<const float4*>(g.gam + (size_t)(smp0 + j) * g.Kg + kc + 4 * q);
      } else {
        const int j = c >> 4, part = (c >> 3) & 1, q = c & 7;
        const int k = kc + 4 * q;
        const bool top = kc < g.N;
        // B_re = [Gr ; -Gi], B_im = [Gi ; Gr] over K = 2 Np
        const int src = part ? (top ? k + g.N : k - g.N) : k;
        float4 v = *reinterpret_cast<const float4*>(g.gam + (size_t)(smp0 + j) * g.Kg + src);
        if (!part && !top) {
          v.x = -v.x;
          v.y = -v.y;
          v.z = -v.z;
          v.w = -v.w;
        }
        *rb[h] = v;
      }
    }
  };
  auto put_b = [&](int buf, int c, float4 v) {
    int col, q;
    if (!CPLX) {
      col = c >> 3;
      q = c & 7;
    } else {
      const int j = c >> 4, part = (c >> 3) & 1;
      q = c & 7;
      col = j + 32 * part + (j >= 32 ? 32 : 0);
    }
    const float f[4] = {v.x, v.y, v.z, v.w};
    uint32_t hb[4], lb[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      hb[e] = bf16_rn(f[e]);
      lb[e] = bf16_rn(f[e] - __uint_as_float(hb[e] << 16));
    }
    *reinterpret_cast<uint2*>(&Bh[buf][swq(col, q >> 1) + 4 * (q & 1)]) =
        make_uint2(hb[0] | (hb[1] << 16), hb[2] | (hb[3] << 16));
    *reinterpret_cast<uint2*>(&Bl[buf][swq(col, q >> 1) + 4 * (q & 1)]) =
        make_uint2(lb[0] | (lb[1] << 16), lb[2] | (lb[3] << 16));
  };
  auto store_chunk = [&](int buf) {
    const int s0 = tid >> 2, q0 = tid & 3;
    const int s1 = (tid + 256) >> 2;
    *reinterpret_cast<uint4*>(&Ah[buf][swq(s0, q0)]) = rah0;
    *reinterpret_cast<uint4*>(&Ah[buf][swq(s1, q0)]) = rah1;
    *reinterpret_cast<uint4*>(&Al[buf][swq(s0, q0)]) = ral0;
    *reinterpret_cast<uint4*>(&Al[buf][swq(s1, q0)]) = ral1;
    put_b(buf, tid, rb0);
    put_b(buf, tid + 256, rb1);
    put_b(buf, tid + 512, rb2);
    put_b(buf, tid + 768, rb3);
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
  for (int kc = 0; kc < K; kc += BK) {
    const bool more = kc + BK < K;
    if (more) load_chunk(kc + BK);
#pragma unroll
    for (int ks = 0; ks < BK; ks += 16) {
      const int ko = ks + 8 * kh;
      const bf16x8 ah0 = *reinterpret_cast<const bf16x8*>(&Ah[buf][swq(wm + li, ko >> 3)]);
      const bf16x8 ah1 = *reinterpret_cast<const bf16x8*>(&Ah[buf][swq(wm + 32 + li, ko >> 3)]);
      const bf16x8 al0 = *reinterpret_cast<const bf16x8*>(&Al[buf][swq(wm + li, ko >> 3)]);
      const bf16x8 al1 = *reinterpret_cast<const bf16x8*>(&Al[buf][swq(wm + 32 + li, ko >> 3)]);
      const bf16x8 bh0 = *reinterpret_cast<const bf16x8*>(&Bh[buf][swq(wn + li, ko >> 3)]);
      const bf16x8 bh1 = *reinterpret_cast<const bf16x8*>(&Bh[buf][swq(wn + 32 + li, ko >> 3)]);
      const bf16x8 bl0 = *reinterpret_cast<const bf16x8*>(&Bl[buf][swq(wn + li, ko >> 3)]);
      const bf16x8 bl1 = *reinterpret_cast<const bf16x8*>(&Bl[buf][swq(wn + 32 + li, ko >> 3)]);
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
__global__ __launch_bounds__(256, 2) void weights_bf16_kernel(WArgsB a) {
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



// 256-thread launch; with events, stamped by the dispatch itself.
template <typename K, typename... A>
void launch256(K kernel, dim3 grid, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1, A... args) {
  if (ev0)
    hipExtLaunchKernelGGL(kernel, grid, dim3(256), 0, st, ev0, ev1, 0, args...);
  else
    hipLaunchKernelGGL(kernel, grid, dim3(256), 0, st, args...);
}

}  // namespace

void launch_weights(const Dims& d, const Work& w, const void* ubulk_t,
                    const void* ubf, int S, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1,
                    unsigned long long* stamp) {
  WArgs g = make_wargs(d, w, ubulk_t);
  g.stamp = stamp;
  const int s_round = (S + SAMPLE_PAD - 1) / SAMPLE_PAD * SAMPLE_PAD;
  if (d.bf16) {
    WArgsB b;
    b.o = g;
    b.uh = static_cast<const uint16_t*>(ubf);
    b.ul = b.uh + (size_t)d.Kg * d.L_pad;
    if (d.cplx)
      launch256(weights_bf16_kernel<true>, dim3(d.L_pad / MT, s_round / (NT / 2)), st, ev0, ev1, b);
    else
      launch256(weights_bf16_kernel<false>, dim3(d.L_pad / MT, s_round / NT), st, ev0, ev1, b);
    return;
  }
  launch_weights_variant(d, g, s_round, tile_choice(d, s_round), st, ev0, ev1);
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
      case 4: launch256(weights_kernel<true, 128, 128, 16, 4>, grid, st, ev0, ev1, g); break;
      case 5: launch256(weights_kernel<true, 64, 128, 16, 6>, grid, st, ev0, ev1, g); break;
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
