// Batched all-site weight evaluation (the "2Lk inner products" of the cost
// count after Eq. (3)) for S samples sharing one U, as one contraction per
// step on the FP32 matrix cores:
//
//   V = U . Gamma      (L_pad x K) . (K x S),  w(x, s) = |V(x, s)|^2
//
// Real U: K = N and Gamma[s] is the dense N-vector of step t (1 at m_t,
// -beta at m_<t).  Complex U is embedded as a real product: A = [Ur | Ui]
// (L x 2N) and two output columns per sample, B_re = [Gr ; -Gi] and
// B_im = [Gi ; Gr], so V_re = Ur Gr - Ui Gi and V_im = Ur Gi + Ui Gr (the
// bilinear u^T h of Eq. (3)); w = V_re^2 + V_im^2.
//
// Epilogue (fused): occupied sites get weight 0; w is stored in float32
// [S][L_pad]; float64 sums of each aligned 32-site block are stored in
// [S][L_pad/32] for the inverse-CDF scan.
//
// Tiling: 256 threads (4 wavefronts), workgroup tile 128 sites x 128 GEMM
// columns, each wavefront 64 x 64 as 2 x 2 v_mfma_f32_32x32x2f32 tiles;
// K in chunks of 16 through double-buffered LDS.  Every output element is
// accumulated over K in the same fixed order whatever its tile, so results do
// not depend on the batch size or on which tile a sample falls in.
#include "ffs_internal.h"

namespace ffsk {

typedef float floatx16 __attribute__((ext_vector_type(16)));

namespace {

constexpr int MT = 128;  // sites per workgroup tile
constexpr int NT = 128;  // GEMM columns per workgroup tile
constexpr int KC = 16;   // K chunk

struct WArgs {
  const float* ut;       // [K][L_pad] k-major bulk U (complex: Ur rows, then Ui)
  const float* gam;      // [S_pad][Kg]
  const uint32_t* occ;   // [S_pad][L_pad/32]
  float* wh;             // [S_pad][L_pad]
  double* bsum;          // [S_pad][L_pad/32]
  int L_pad, N, Kg, S_pad;
};

template <bool CPLX>
__global__ __launch_bounds__(256) void weights_kernel(WArgs g) {
  __shared__ float As[2][KC][MT];
  __shared__ float Bs[2][KC][NT + 4];
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int wm = (wave & 1) * 64;   // wave's site offset in the tile
  const int wn = (wave >> 1) * 64;  // wave's GEMM-column offset in the tile
  const int site0 = blockIdx.x * MT;
  // GEMM columns of this tile: real -> samples col0..col0+127;
  // complex -> samples smp0..smp0+63, laid out per wavefront as
  // [re(32 samples) | im(same 32 samples)].
  const int K = CPLX ? 2 * g.N : g.N;
  const int smp0 = blockIdx.y * (CPLX ? NT / 2 : NT);

  // global -> register staging
  float4 ra[2];
  float bre[CPLX ? 4 : 8];
  float bim[CPLX ? 4 : 1];
  (void)bim;

  auto load_chunk = [&](int kc) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int kk = (tid >> 5) + 8 * h;
      const int col = (tid & 31) * 4;
      ra[h] = *reinterpret_cast<const float4*>(g.ut + (size_t)(kc + kk) * g.L_pad + site0 + col);
    }
    if (!CPLX) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int j = (tid >> 2) + 64 * h;
        const int kq = tid & 3;
        const float4 v = *reinterpret_cast<const float4*>(g.gam + (size_t)(smp0 + j) * g.Kg + kc + 4 * kq);
        bre[4 * h + 0] = v.x; bre[4 * h + 1] = v.y; bre[4 * h + 2] = v.z; bre[4 * h + 3] = v.w;
      }
    } else {
      const int j = tid >> 2;  // sample 0..63 within the tile
      const int kq = tid & 3;
      const int k = kc + 4 * kq;
      // re column: sign * gam[k]; im column: gam[(k + N) mod 2N]
      const float sg = (kc < g.N) ? 1.0f : -1.0f;
      const int kim = (kc < g.N) ? k + g.N : k - g.N;
      const float4 v = *reinterpret_cast<const float4*>(g.gam + (size_t)(smp0 + j) * g.Kg + k);
      const float4 w = *reinterpret_cast<const float4*>(g.gam + (size_t)(smp0 + j) * g.Kg + kim);
      bre[0] = sg * v.x; bre[1] = sg * v.y; bre[2] = sg * v.z; bre[3] = sg * v.w;
      bim[0] = w.x; bim[1] = w.y; bim[2] = w.z; bim[3] = w.w;
    }
  };
  auto store_chunk = [&](int buf) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int kk = (tid >> 5) + 8 * h;
      const int col = (tid & 31) * 4;
      *reinterpret_cast<float4*>(&As[buf][kk][col]) = ra[h];
    }
    if (!CPLX) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int j = (tid >> 2) + 64 * h;
        const int kq = tid & 3;
#pragma unroll
        for (int c = 0; c < 4; ++c) Bs[buf][4 * kq + c][j] = bre[4 * h + c];
      }
    } else {
      const int j = tid >> 2;
      const int kq = tid & 3;
      const int cre = 64 * (j >> 5) + (j & 31);
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        Bs[buf][4 * kq + c][cre] = bre[c];
        Bs[buf][4 * kq + c][cre + 32] = bim[c];
      }
    }
  };

  floatx16 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;

  load_chunk(0);
  store_chunk(0);
  __syncthreads();
  int buf = 0;
  for (int kc = 0; kc < K; kc += KC) {
    const bool more = kc + KC < K;
    if (more) load_chunk(kc + KC);
#pragma unroll
    for (int kk = 0; kk < KC; kk += 2) {
      const int kr = kk + (lane >> 5);
      const int li = lane & 31;
      const float a0 = As[buf][kr][wm + li];
      const float a1 = As[buf][kr][wm + 32 + li];
      const float b0 = Bs[buf][kr][wn + li];
      const float b1 = Bs[buf][kr][wn + 32 + li];
      acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b1, acc[1][1], 0, 0, 0);
    }
    if (more) {
      store_chunk(buf ^ 1);
      __syncthreads();
      buf ^= 1;
    }
  }

  // ---- epilogue -------------------------------------------------------------
  // C layout of a 32x32 tile: lane l, register r -> column l%32,
  // row 8*(r/4) + 4*(l/32) + r%4.
  const int li = lane & 31, hf = lane >> 5;
  const int nblk = g.L_pad / 32;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int sb = site0 + wm + 32 * i;  // first site of this 32-site block
    const int blk = sb >> 5;
#pragma unroll
    for (int jt = 0; jt < (CPLX ? 1 : 2); ++jt) {
      const int smp = CPLX ? (smp0 + (wn >> 1) + li) : (smp0 + wn + 32 * jt + li);
      const uint32_t occw = g.occ[(size_t)smp * nblk + blk];
      float w[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = 8 * (r >> 2) + 4 * hf + (r & 3);
        float v;
        if (CPLX) {
          const float re = acc[i][0][r], im = acc[i][1][r];
          v = re * re + im * im;
        } else {
          const float re = acc[i][jt][r];
          v = re * re;
        }
        w[r] = ((occw >> row) & 1u) ? 0.0f : v;
      }
      float* dst = g.wh + (size_t)smp * g.L_pad + sb + 4 * hf;
      double part = 0.0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        *reinterpret_cast<float4*>(dst + 8 * q) =
            make_float4(w[4 * q], w[4 * q + 1], w[4 * q + 2], w[4 * q + 3]);
#pragma unroll
        for (int c = 0; c < 4; ++c) part += (double)w[4 * q + c];
      }
      const double other = __shfl_xor(part, 32, 64);
      const double tot = (hf == 0) ? part + other : other + part;
      if (hf == 0) g.bsum[(size_t)smp * nblk + blk] = tot;
    }
  }
}

}  // namespace

void launch_weights(const Dims& d, const Work& w, const void* ubulk_t, int S,
                    hipStream_t st) {
  WArgs g;
  g.ut = static_cast<const float*>(ubulk_t);
  g.gam = static_cast<const float*>(w.gam);
  g.occ = w.occ;
  g.wh = static_cast<float*>(w.wh);
  g.bsum = w.bsum;
  g.L_pad = d.L_pad;
  g.N = d.Np;
  g.Kg = d.Kg;
  g.S_pad = w.S_pad;
  const int s_round = (S + SAMPLE_PAD - 1) / SAMPLE_PAD * SAMPLE_PAD;
  if (d.cplx) {
    dim3 grid(d.L_pad / MT, s_round / (NT / 2));
    hipLaunchKernelGGL(weights_kernel<true>, grid, dim3(256), 0, st, g);
  } else {
    dim3 grid(d.L_pad / MT, s_round / NT);
    hipLaunchKernelGGL(weights_kernel<false>, grid, dim3(256), 0, st, g);
  }
}

}  // namespace ffsk
