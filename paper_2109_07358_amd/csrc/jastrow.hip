// Slater-Jastrow reweighting (SI S-5, Eq. (S8)): configurations x drawn from
// the free-fermion ensemble |psi_0(x)|^2 estimate expectations in the
// Jastrow-correlated state psi_J = J psi_0 as <O> = <J^2 o_L>_0 / <J^2>_0.
// For spin-1/2 fermions a configuration is a pair (x_up, x_dn) of draws
// (each row of x one sample; -1 entries are empty slots); J is diagonal in
// the position basis, with
//   log J^2(x) = -V D(x) - sum_{i,j} v_ij n_i n_j  [+ a caller's log-weight]
// where D = #sites holding both spins (the Gutzwiller factor of the main
// text, J = exp(-V/2 sum_i n_i,up n_i,dn)) and n_i = n_i,up + n_i,dn (the
// general two-body density form of SI S-5, v an L x L matrix).  The
// observables are diagonal, so o_L(x) is their value at x: the site
// densities <n_i> and the double occupancy <D>.
//
// Kernels, all float64 and in a fixed summation order:
//   jastrow_counts_kernel, jastrow_pair_mma_kernel (the pair term when L is
//                        at most 16 particles' worth of sites): per sample
//                        the site counts n, then sum_ij n_i v_ij n_j =
//                        sum_j (N v)[s, j] n_j for a chunk of samples as one
//                        product on the FP64 matrix cores (N the counts, one
//                        row per sample), reduced per 64-site tile;
//   jastrow_logw_kernel  one workgroup per sample: up-spin occupancy bitmap
//                        in LDS, D by lookups of the down spins, the pair sum
//                        split over threads by first particle, then reduced
//                        in a fixed tree;
//   jastrow_max_kernel   m = max_s log J^2 (weights w_s = exp(logw_s - m));
//   jastrow_accum_kernel (site tile, group of 256 samples) per workgroup:
//                        samples in order, up then down spins, adding w_s to
//                        an LDS tile of the density (no two threads touch one
//                        site within a phase); group sums of w, w^2, w D, D;
//   jastrow_final_kernel sums the groups in order and normalises.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>

#include "../../include/ffs.h"
#include "ffs_internal.h"

using namespace ffsk;

namespace {

constexpr int kJTile = 1024;   // sites per accumulation tile
constexpr int kJGroup = 256;   // samples per accumulation group
constexpr int kJMaxL = 65536;

__device__ inline double block_sum_256(double v, double* red) {
  // fixed order: lanes by xor butterfly, then the four wavefronts in order
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  return ((red[0] + red[1]) + red[2]) + red[3];
}

// Samples s_base + blockIdx.x.  pp (nullable): the pair term as npp
// per-tile partial sums per sample (row blockIdx.x), else gathered from vmat.
__global__ __launch_bounds__(256) void jastrow_logw_kernel(
    const int32_t* xu, int ku, const int32_t* xd, int kd, int L, double V, const double* vmat,
    const double* pp, int npp, int s_base, const double* extra, double* logw, int32_t* dcount,
    int32_t* status) {
  __shared__ uint32_t bits[kJMaxL / 32];
  __shared__ double red[4];
  __shared__ int dsum[4];
  const int s = s_base + blockIdx.x, tid = threadIdx.x;
  const int32_t* up = xu + (size_t)s * ku;
  const int32_t* dn = xd ? xd + (size_t)s * kd : nullptr;
  const int nw = (L + 31) / 32;
  for (int i = tid; i < nw; i += 256) bits[i] = 0u;
  __syncthreads();
  bool bad = false;
  for (int a = tid; a < ku; a += 256) {
    const int y = up[a];
    if (y >= L || y < -1) bad = true;
    else if (y >= 0) atomicOr(&bits[y >> 5], 1u << (y & 31));
  }
  __syncthreads();
  int d = 0;
  for (int a = tid; a < kd; a += 256) {
    const int y = dn[a];
    if (y >= L || y < -1) bad = true;
    else if (y >= 0 && ((bits[y >> 5] >> (y & 31)) & 1u)) ++d;
  }
  if (bad) atomicOr(status, (int)DEV_BADCOLS);
  // D: wavefront sums, then the four wavefronts in order
  for (int o = 32; o >= 1; o >>= 1) d += __shfl_xor(d, o, 64);
  if ((tid & 63) == 0) dsum[tid >> 6] = d;
  __syncthreads();
  const int D = ((dsum[0] + dsum[1]) + dsum[2]) + dsum[3];
  double pair = 0.0;
  if (pp) {
    if (tid == 0) {
      const double* row = pp + (size_t)blockIdx.x * npp;
      for (int t = 0; t < npp; ++t) pair += row[t];
    }
  } else if (vmat) {
    // sum over ordered particle pairs (a, b), both spins, empty slots skipped
    const int P = ku + kd;
    for (int a = tid; a < P; a += 256) {
      const int ya = a < ku ? up[a] : dn[a - ku];
      if (ya < 0 || ya >= L) continue;
      const double* row = vmat + (size_t)ya * L;
      double acc = 0.0;
      for (int b = 0; b < P; ++b) {
        const int yb = b < ku ? up[b] : dn[b - ku];
        if (yb >= 0 && yb < L) acc += row[yb];
      }
      pair += acc;
    }
    pair = block_sum_256(pair, red);
  }
  if (tid == 0) {
    double lw = -V * (double)D - pair;
    if (extra) lw += extra[s];
    logw[s] = lw;
    dcount[s] = D;
  }
}

// Site counts of samples s_base + r (r < nr; rows nr..gridDim.x-1 zero):
// nm[r][y] = number of particles (both spins) on site y, nm of row stride Lp
// with zeros past L.  Sites outside [0, L) are skipped here (the log-weight
// kernel reports them).  Adding 1.0 is exact in any order.
__global__ __launch_bounds__(256) void jastrow_counts_kernel(
    const int32_t* xu, int ku, const int32_t* xd, int kd, int L, int Lp, int s_base, int nr,
    double* nm) {
  const int r = blockIdx.x, tid = threadIdx.x;
  double* row = nm + (size_t)r * Lp;
  for (int i = tid; i < Lp; i += 256) row[i] = 0.0;
  __syncthreads();
  if (r >= nr) return;
  const int s = s_base + r;
  for (int a = tid; a < ku + kd; a += 256) {
    const int y = a < ku ? xu[(size_t)s * ku + a] : xd[(size_t)s * kd + a - ku];
    if (y >= 0 && y < L) atomicAdd(&row[y], 1.0);
  }
}

typedef double doublex4 __attribute__((ext_vector_type(4)));

// W = N v for samples r0..r0+63 (rows of nm) and sites j0..j0+63, one
// wavefront as 4 x 4 tiles of v_mfma_f64_16x16x4f64 over k in groups of
// 16 (k = k0 + 4 (l / 16) + j for MFMA j, the same in both operands); then
// pp[r][blockIdx.x] = sum_j W[r][j] nm[r][j] over the tile's 64 sites
// (per lane its four 16-site tiles in order, then the 16 lanes of the row
// by a fixed xor butterfly).  MFMA layout: A[l%16][l/16], B[l/16][l%16],
// register q of lane l = D[l/16 + 4q][l%16].
__global__ __launch_bounds__(64, 2) void jastrow_pair_mma_kernel(const double* nm, int Lp,
                                                                 const double* v, int L,
                                                                 double* pp) {
  const int lane = threadIdx.x, li = lane & 15, lg = lane >> 4;
  const int j0 = blockIdx.x * 64, r0 = blockIdx.y * 64;
  const int npp = Lp / 64;
  doublex4 acc[4][4];
#pragma unroll
  for (int rt = 0; rt < 4; ++rt)
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) acc[rt][ct] = doublex4{0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < Lp; k0 += 16) {
    double a[4][4], b[4][4];
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) {
      const doublex4 x =
          *reinterpret_cast<const doublex4*>(nm + (size_t)(r0 + 16 * rt + li) * Lp + k0 + 4 * lg);
      a[rt][0] = x.x;
      a[rt][1] = x.y;
      a[rt][2] = x.z;
      a[rt][3] = x.w;
    }
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      const int k = k0 + 4 * lg + jj;
#pragma unroll
      for (int ct = 0; ct < 4; ++ct) {
        const int j = j0 + 16 * ct + li;
        b[ct][jj] = (k < L && j < L) ? v[(size_t)k * L + j] : 0.0;
      }
    }
#pragma unroll
    for (int jj = 0; jj < 4; ++jj)
#pragma unroll
      for (int rt = 0; rt < 4; ++rt)
#pragma unroll
        for (int ct = 0; ct < 4; ++ct)
          acc[rt][ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[rt][jj], b[ct][jj], acc[rt][ct], 0, 0, 0);
  }
#pragma unroll
  for (int rt = 0; rt < 4; ++rt)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = r0 + 16 * rt + lg + 4 * q;
      const double* nrow = nm + (size_t)r * Lp + j0 + li;
      double sum = 0.0;
#pragma unroll
      for (int ct = 0; ct < 4; ++ct) sum += acc[rt][ct][q] * nrow[16 * ct];
      for (int o = 1; o < 16; o <<= 1) sum += __shfl_xor(sum, o, 64);
      if (li == 0) pp[(size_t)r * npp + blockIdx.x] = sum;
    }
}

__global__ __launch_bounds__(256) void jastrow_max_kernel(const double* logw, int n, double* out) {
  __shared__ double red[256];
  double m = -INFINITY;
  for (int i = threadIdx.x; i < n; i += 256) m = fmax(m, logw[i]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int o = 128; o >= 1; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

// grid (tiles, groups).  part: [groups][L]; gsum: [groups][4] = sum w,
// sum w^2, sum w D, sum D.
__global__ __launch_bounds__(256) void jastrow_accum_kernel(
    const int32_t* xu, int ku, const int32_t* xd, int kd, int n, int L, const double* logw,
    const int32_t* dcount, const double* mx, double* part, double* gsum) {
  __shared__ double acc[kJTile];
  const int i0 = blockIdx.x * kJTile, g = blockIdx.y, tid = threadIdx.x;
  const int s0 = g * kJGroup, s1 = min(n, s0 + kJGroup);
  const double m = mx[0];
  for (int i = tid; i < kJTile; i += 256) acc[i] = 0.0;
  __syncthreads();
  for (int s = s0; s < s1; ++s) {
    const double w = exp(logw[s] - m);
    const int32_t* up = xu + (size_t)s * ku;
    for (int a = tid; a < ku; a += 256) {
      const int y = up[a] - i0;
      if (up[a] >= 0 && y >= 0 && y < kJTile) acc[y] += w;
    }
    __syncthreads();
    if (xd) {
      const int32_t* dn = xd + (size_t)s * kd;
      for (int a = tid; a < kd; a += 256) {
        const int y = dn[a] - i0;
        if (dn[a] >= 0 && y >= 0 && y < kJTile) acc[y] += w;
      }
      __syncthreads();
    }
  }
  for (int i = tid; i < kJTile; i += 256)
    if (i0 + i < L) part[(size_t)g * L + i0 + i] = acc[i];
  if (blockIdx.x == 0 && tid == 0) {
    double sw = 0.0, sw2 = 0.0, swd = 0.0, sd = 0.0;
    for (int s = s0; s < s1; ++s) {
      const double w = exp(logw[s] - m);
      sw += w;
      sw2 += w * w;
      swd += w * (double)dcount[s];
      sd += (double)dcount[s];
    }
    gsum[g * 4 + 0] = sw;
    gsum[g * 4 + 1] = sw2;
    gsum[g * 4 + 2] = swd;
    gsum[g * 4 + 3] = sd;
  }
}

// density[i] = sum_g part[g][i] / sum w; summary as documented in ffs.h.
__global__ void jastrow_final_kernel(const double* part, const double* gsum, int groups, int n,
                                     int L, const double* mx, double* density, double* summary) {
  __shared__ double tot[4];
  if (threadIdx.x == 0) {
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    for (int g = 0; g < groups; ++g)
      for (int c = 0; c < 4; ++c) a[c] += gsum[g * 4 + c];
    for (int c = 0; c < 4; ++c) tot[c] = a[c];
    if (blockIdx.x == 0) {
      summary[0] = a[2] / a[0];           // <D>_J
      summary[1] = a[3] / (double)n;      // <D>_0
      summary[2] = a[0];                  // sum w
      summary[3] = a[1];                  // sum w^2
      summary[4] = a[0] * a[0] / a[1];    // effective sample size
      summary[5] = mx[0];                 // the shift m
    }
  }
  __syncthreads();
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < L) {
    double acc = 0.0;
    for (int g = 0; g < groups; ++g) acc += part[(size_t)g * L + i];
    density[i] = acc / tot[0];
  }
}

#define J_HIP(call)                                                         \
  do {                                                                      \
    hipError_t e_ = (call);                                                 \
    if (e_ != hipSuccess) {                                                 \
      set_error(FFS_ERR_HIP, hipGetErrorString(e_));                        \
      return FFS_ERR_HIP;                                                   \
    }                                                                       \
  } while (0)

}  // namespace

extern "C" ffs_status ffs_jastrow_estimate(const int32_t* x_up_dev, int64_t k_up,
                                           const int32_t* x_dn_dev, int64_t k_dn,
                                           int64_t n_samples, int64_t L, double V,
                                           const double* vmat_dev, const double* extra_logw_dev,
                                           double* logw_dev, double* density_dev,
                                           double* summary_dev, void* stream) {
  if (!x_up_dev || !logw_dev || !density_dev || !summary_dev)
    return (ffs_status)set_error(FFS_ERR_INVALID_ARG, "NULL x_up_dev or output");
  if (k_up < 1 || k_dn < 0 || (k_dn > 0 && !x_dn_dev) || n_samples < 1 || L < 1)
    return (ffs_status)set_error(FFS_ERR_INVALID_ARG, "need k_up >= 1, k_dn >= 0, n >= 1, L >= 1");
  if (L > kJMaxL || k_up > 65536 || k_dn > 65536 || n_samples > (int64_t)1 << 24)
    return (ffs_status)set_error(FFS_ERR_UNSUPPORTED, "L above 65536 or sizes too large");
  if (!isfinite(V)) return (ffs_status)set_error(FFS_ERR_INVALID_ARG, "V not finite");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int n = (int)n_samples, Li = (int)L, ku = (int)k_up, kd = (int)k_dn;
  const int groups = (n + kJGroup - 1) / kJGroup, tiles = (Li + kJTile - 1) / kJTile;
  const size_t b_part = (size_t)groups * L * 8, b_g = (size_t)groups * 32;
  // Pair term on the matrix cores when the dense L^2 product per sample is
  // cheaper than the P^2 scattered reads of v (P = ku + kd particles): the
  // product runs near the FP64 MFMA rate, the reads at a few 10^10 per s.
  const int P = ku + kd;
  const bool mma = vmat_dev && (int64_t)Li <= 16 * (int64_t)P;
  const int Lp = (Li + 63) / 64 * 64;
  int chunk = n;
  size_t b_nm = 0, b_pp = 0;
  if (mma) {  // samples per product: counts and partial sums within 256 MB
    const size_t per_row = (size_t)Lp * 8 + (size_t)(Lp / 64) * 8;
    const int64_t rows = (int64_t)((256ull << 20) / per_row) / 64 * 64;
    chunk = (int)std::min<int64_t>(n, std::max<int64_t>(64, rows));
    const size_t cp = (size_t)(chunk + 63) / 64 * 64;
    b_nm = cp * Lp * 8;
    b_pp = cp * (Lp / 64) * 8;
  }
  const size_t b_base = (b_part + b_g + (size_t)n * 4 + 512 + 255) / 256 * 256;
  char* buf = nullptr;
  J_HIP(hipMallocAsync((void**)&buf, b_base + b_nm + b_pp, st));
  double* nm = mma ? reinterpret_cast<double*>(buf + b_base) : nullptr;
  double* pp = mma ? reinterpret_cast<double*>(buf + b_base + b_nm) : nullptr;
  double* part = reinterpret_cast<double*>(buf);
  double* gsum = reinterpret_cast<double*>(buf + b_part);
  int32_t* dcount = reinterpret_cast<int32_t*>(buf + b_part + b_g);
  double* mx = reinterpret_cast<double*>(buf + b_part + b_g + (((size_t)n * 4 + 255) / 256) * 256);
  int32_t* status = reinterpret_cast<int32_t*>(mx + 8);
  J_HIP(hipMemsetAsync(status, 0, 4, st));
  const int32_t* xd = kd > 0 ? x_dn_dev : nullptr;
  for (int s0 = 0; s0 < n; s0 += chunk) {
    const int nc = std::min(chunk, n - s0), ncp = (nc + 63) / 64 * 64;
    if (mma) {
      hipLaunchKernelGGL(jastrow_counts_kernel, dim3(ncp), dim3(256), 0, st, x_up_dev, ku, xd, kd,
                         Li, Lp, s0, nc, nm);
      hipLaunchKernelGGL(jastrow_pair_mma_kernel, dim3(Lp / 64, ncp / 64), dim3(64), 0, st, nm,
                         Lp, vmat_dev, Li, pp);
    }
    hipLaunchKernelGGL(jastrow_logw_kernel, dim3(nc), dim3(256), 0, st, x_up_dev, ku, xd, kd, Li,
                       V, vmat_dev, pp, Lp / 64, s0, extra_logw_dev, logw_dev, dcount, status);
  }
  hipLaunchKernelGGL(jastrow_max_kernel, dim3(1), dim3(256), 0, st, logw_dev, n, mx);
  hipLaunchKernelGGL(jastrow_accum_kernel, dim3(tiles, groups), dim3(256), 0, st, x_up_dev, ku,
                     kd > 0 ? x_dn_dev : nullptr, kd, n, Li, logw_dev, dcount, mx, part, gsum);
  hipLaunchKernelGGL(jastrow_final_kernel, dim3((Li + 255) / 256), dim3(256), 0, st, part, gsum,
                     groups, n, Li, mx, density_dev, summary_dev);
  int h = 0;
  J_HIP(hipMemcpyAsync(&h, status, 4, hipMemcpyDeviceToHost, st));
  J_HIP(hipFreeAsync(buf, st));
  J_HIP(hipStreamSynchronize(st));
  J_HIP(hipGetLastError());
  if (h) return (ffs_status)set_error(FFS_ERR_INVALID_ARG, "site outside [-1, L) in x");
  return FFS_OK;
}
