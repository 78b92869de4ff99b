// Device front end of DPP subset selection (the paper's application of the
// sampler to text summarisation): an L-ensemble kernel C = B B^T built from
// L feature vectors b_i (rows of B, L x d) is diagonalised through its d x d
// dual B^T B, each eigenvector is then kept at random -- with probability
// lambda / (lambda + 1) for the DPP the paper uses, or as a fixed-size
// subset for a k-DPP (Kulesza and Taskar's elementary-symmetric-polynomial
// selection) -- and the kept eigenvectors are the orthonormal columns U on
// which the fermion sampler draws the items (ffs_sample_subsets).
//
// Kernels, all float64:
//   gram_kernel      C = B^T B, 32 x 32 tiles, each entry summed over the L
//                    rows in ascending order (C comes out exactly symmetric);
//   jacobi_round_kernel
//                    cyclic two-sided Jacobi on C, one launch per
//                    round-robin round: the d/2 disjoint rotations of the
//                    round are formed from the matrix before it, applied to
//                    its rows, then to its columns (2 x 2 blocks, one thread
//                    each, into a second buffer) and to the accumulated
//                    eigenvectors; a rotation is skipped when |c_pq| <= tol
//                    sqrt(|c_pp c_qq|) (tol = 1e-14), the rotated pair's
//                    off-diagonal entries are set to zero, and the sweeps end
//                    when a whole sweep skips every rotation;
//   order_kernel     eigenvalues ascending (ties by index), each eigenvector
//                    signed so that its largest-magnitude entry (first one on
//                    ties) is positive;
//   project_kernel   U = B W Lambda^{-1/2} (the eigenvectors of B B^T with
//                    nonzero eigenvalue, orthonormal);
//   esp_kernel       table e_m(lambda_0..lambda_{j-1}) of elementary
//                    symmetric polynomials of the eigenvalues divided by the
//                    largest one, rows m = 0..k (recurrence over j, products
//                    and sums rounded separately);
//   kdpp_kernel /    one thread per sample: eigenvalues scanned from the last
//   dpp_kernel       with one Philox uniform each (stream word 1, step = the
//                    eigenvalue's index), kept by the k-DPP rule or with
//                    probability lambda / (lambda + 1).
#include <hip/hip_runtime.h>
#include <math.h>

#include <vector>

#include "../../include/ffs.h"
#include "ffs_internal.h"

using namespace ffsk;

namespace {

constexpr int kDppMaxD = 512;     // dual dimension of the eigendecomposition
constexpr int kMaxSweeps = 60;
constexpr uint32_t kSelectStream = 1u;

__global__ __launch_bounds__(256) void gram_kernel(const double* B, int L, int d, double* C) {
  __shared__ double bi[64][33], bj[64][33];
  const int i0 = blockIdx.y * 32, j0 = blockIdx.x * 32;
  const int tid = threadIdx.x, ti = tid >> 4, tj = tid & 15;
  double acc[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
  for (int l0 = 0; l0 < L; l0 += 64) {
    for (int e = tid; e < 64 * 32; e += 256) {
      const int r = e >> 5, c = e & 31, l = l0 + r;
      bi[r][c] = (l < L && i0 + c < d) ? B[(size_t)l * d + i0 + c] : 0.0;
      bj[r][c] = (l < L && j0 + c < d) ? B[(size_t)l * d + j0 + c] : 0.0;
    }
    __syncthreads();
    for (int r = 0; r < 64; ++r)
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = fma(bi[r][2 * ti + a], bj[r][2 * tj + b], acc[a][b]);
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int i = i0 + 2 * ti + a, j = j0 + 2 * tj + b;
      if (i < d && j < d) C[(size_t)i * d + j] = acc[a][b];
    }
}

// ---- cyclic two-sided Jacobi, one launch per round, spread over the chip ----
// Round r of the circle-method schedule pairs (n-1, r) and ((r+k) mod (n-1),
// (r-k) mod (n-1)), k = 1..n/2-1 (n = d rounded up to even, index d a bye).
__device__ inline void jacobi_pair(int k, int r, int n, int* p, int* q) {
  const int a = k == 0 ? n - 1 : (r + k) % (n - 1);
  const int b = k == 0 ? r : (r - k + (n - 1)) % (n - 1);
  *p = a < b ? a : b;
  *q = a < b ? b : a;
}

// Rotation of pair (p, q) from the matrix before the round: skipped (false,
// c = 1, s = 0) when |a_pq| <= tol sqrt(|a_pp a_qq|), else the angle that
// zeroes a_pq (t = sign(theta) / (|theta| + sqrt(theta^2 + 1)), theta =
// (a_qq - a_pp) / (2 a_pq)).
__device__ inline bool jacobi_rot(const double* A, int d, int p, int q, double tol, double* c,
                                  double* s) {
  *c = 1.0;
  *s = 0.0;
  if (q >= d) return false;
  const double apq = A[(size_t)p * d + q];
  const double app = A[(size_t)p * d + p], aqq = A[(size_t)q * d + q];
  if (!(fabs(apq) > tol * sqrt(fabs(app * aqq)))) return false;
  const double theta = (aqq - app) / (2.0 * apq);
  const double at = fabs(theta);
  const double t = (at > 1e150 ? 0.5 / at : 1.0 / (at + sqrt(theta * theta + 1.0)));
  const double ts = theta < 0.0 ? -t : t;
  *c = 1.0 / sqrt(ts * ts + 1.0);
  *s = ts * (*c);
  return true;
}

// One round: thread (a, b) < np^2 writes the rotated 2 x 2 block of row pair a
// and column pair b into Aout -- rows first (J^T A), then columns (. J, which
// sets the rotated pair's own off-diagonal entries to zero) -- every rotation
// formed from Ain, the matrix before the round; the next d * np threads
// rotate the column pairs of V in place.
// Each element is written by one thread, so rounds need no barrier inside a
// launch; the launches of a sweep alternate Ain and Aout.
__global__ __launch_bounds__(256) void jacobi_round_kernel(const double* Ain, double* Aout,
                                                           double* V, int d, int n, int r,
                                                           double tol, int* rotated) {
  const int np = n / 2;
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  if (gid < np * np) {
    const int a = gid / np, b = gid - (gid / np) * np;
    int pa, qa, pb, qb;
    jacobi_pair(a, r, n, &pa, &qa);
    jacobi_pair(b, r, n, &pb, &qb);
    double ca, sa, cb, sb;
    const bool ra = jacobi_rot(Ain, d, pa, qa, tol, &ca, &sa);
    const bool rb = jacobi_rot(Ain, d, pb, qb, tol, &cb, &sb);
    if (a == b && ra) *rotated = 1;
    const bool hq = qa < d, hc = qb < d;  // row qa / column qb exist (not a bye)
    // the block, rows (pa, qa) x columns (pb, qb)
    double m00 = Ain[(size_t)pa * d + pb];
    double m01 = hc ? Ain[(size_t)pa * d + qb] : 0.0;
    double m10 = hq ? Ain[(size_t)qa * d + pb] : 0.0;
    double m11 = (hq && hc) ? Ain[(size_t)qa * d + qb] : 0.0;
    if (ra) {  // rows p, q <- J^T A
      const double r00 = ca * m00 - sa * m10, r10 = sa * m00 + ca * m10;
      const double r01 = ca * m01 - sa * m11, r11 = sa * m01 + ca * m11;
      m00 = r00;
      m10 = r10;
      m01 = r01;
      m11 = r11;
    }
    if (rb) {  // columns p, q <- A J; the rotated pair's own off-diagonal is 0
      const double c00 = cb * m00 - sb * m01, c01 = sb * m00 + cb * m01;
      const double c10 = cb * m10 - sb * m11, c11 = sb * m10 + cb * m11;
      m00 = (pa == qb) ? 0.0 : c00;
      m01 = (pa == pb) ? 0.0 : c01;
      m10 = (qa == qb) ? 0.0 : c10;
      m11 = (qa == pb) ? 0.0 : c11;
    }
    Aout[(size_t)pa * d + pb] = m00;
    if (hc) Aout[(size_t)pa * d + qb] = m01;
    if (hq) Aout[(size_t)qa * d + pb] = m10;
    if (hq && hc) Aout[(size_t)qa * d + qb] = m11;
    return;
  }
  const int g2 = gid - np * np;
  if (g2 >= d * np) return;
  const int i = g2 / np, a = g2 - (g2 / np) * np;
  int p, q;
  jacobi_pair(a, r, n, &p, &q);
  double c, s;
  if (!jacobi_rot(Ain, d, p, q, tol, &c, &s)) return;
  const double vp = V[(size_t)i * d + p], vq = V[(size_t)i * d + q];
  V[(size_t)i * d + p] = c * vp - s * vq;
  V[(size_t)i * d + q] = s * vp + c * vq;
}

__global__ void identity_kernel(double* V, int d) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < (size_t)d * d) V[e] = (e / d == e % d) ? 1.0 : 0.0;
}

// Eigenvalue i = A[i][i]; rank = its position in ascending order (ties by
// index).  lam[rank] = A[i][i], W[:, rank] = +-V[:, i].
__global__ void order_kernel(const double* A, const double* V, int d, double* lam, double* W) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d) return;
  const double li = A[(size_t)i * d + i];
  int rank = 0;
  for (int j = 0; j < d; ++j) {
    const double lj = A[(size_t)j * d + j];
    if (lj < li || (lj == li && j < i)) ++rank;
  }
  int rmax = 0;
  double vmax = -1.0;
  for (int r = 0; r < d; ++r) {
    const double v = fabs(V[(size_t)r * d + i]);
    if (v > vmax) {
      vmax = v;
      rmax = r;
    }
  }
  const double sg = V[(size_t)rmax * d + i] < 0.0 ? -1.0 : 1.0;
  lam[rank] = li;
  for (int r = 0; r < d; ++r) W[(size_t)r * d + rank] = sg * V[(size_t)r * d + i];
}

// U[l][j] = (sum_k B[l][k] W[k][j]) / sqrt(lam[j]), k ascending; 32 x 32
// output tile per workgroup, 32-wide k slabs in LDS.
__global__ __launch_bounds__(256) void project_kernel(const double* B, const double* W,
                                                      const double* lam, int L, int d,
                                                      double* U) {
  __shared__ double bt[32][33], wt[32][33];
  const int l0 = blockIdx.x * 32, j0 = blockIdx.y * 32;
  const int tid = threadIdx.x, ti = tid >> 4, tj = tid & 15;
  double acc[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
  for (int k0 = 0; k0 < d; k0 += 32) {
    for (int e = tid; e < 32 * 32; e += 256) {
      const int r = e >> 5, c = e & 31;
      bt[r][c] = (l0 + r < L && k0 + c < d) ? B[(size_t)(l0 + r) * d + k0 + c] : 0.0;
      wt[r][c] = (k0 + r < d && j0 + c < d) ? W[(size_t)(k0 + r) * d + j0 + c] : 0.0;
    }
    __syncthreads();
    for (int k = 0; k < 32; ++k)
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = fma(bt[2 * ti + a][k], wt[k][2 * tj + b], acc[a][b]);
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int l = l0 + 2 * ti + a, j = j0 + 2 * tj + b;
      if (l < L && j < d) U[(size_t)l * d + j] = acc[a][b] / sqrt(lam[j]);
    }
}

// E[m][j] = e_m(mu_0 .. mu_{j-1}), mu = lam / max(lam), m = 0..k, j = 0..d;
// row-major (k+1) x (d+1).  status: 1 if e_k(mu) is not a positive finite
// number or an eigenvalue is negative or not finite.
__global__ void esp_kernel(const double* lam, int d, int k, double* E, int* status) {
#pragma clang fp contract(off)
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double top = 0.0;
  bool bad = false;
  for (int j = 0; j < d; ++j) {
    const double v = lam[j];
    if (!(v >= 0.0) || !isfinite(v)) bad = true;
    if (v > top) top = v;
  }
  const int w = d + 1;
  for (int j = 0; j <= d; ++j) E[j] = 1.0;
  for (int m = 1; m <= k; ++m) {
    E[(size_t)m * w] = 0.0;
    for (int j = 1; j <= d; ++j) {
      const double mu = lam[j - 1] / top;
      const double prod = mu * E[(size_t)(m - 1) * w + j - 1];
      E[(size_t)m * w + j] = E[(size_t)m * w + j - 1] + prod;
    }
  }
  const double ek = E[(size_t)k * w + d];
  if (bad || !(top > 0.0) || !(ek > 0.0) || !isfinite(ek)) *status = 1;
}

// k-DPP eigenvector subset of sample first + s: scan j = d-1 .. 0; with l
// indices still to take, keep j when u_j < mu_j e_{l-1}(mu_<j) / e_l(mu_<=j)
// (always when j + 1 == l).  cols[s][*] ascending.
__global__ void kdpp_kernel(const double* lam, const double* E, int d, int k, uint64_t seed,
                            uint64_t first, int n, int32_t* cols) {
#pragma clang fp contract(off)
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  double top = 0.0;
  for (int j = 0; j < d; ++j)
    if (lam[j] > top) top = lam[j];
  const int w = d + 1;
  int l = k;
  int32_t* out = cols + (size_t)s * k;
  for (int j = d - 1; j >= 0 && l > 0; --j) {
    const double u = uniform53(philox_stream(seed, first + (uint64_t)s, (uint32_t)j, kSelectStream));
    const double mu = lam[j] / top;
    const double num = mu * E[(size_t)(l - 1) * w + j];
    const double p = num / E[(size_t)l * w + j + 1];
    if (j + 1 == l || u < p) {
      out[l - 1] = j;
      --l;
    }
  }
}

// DPP eigenvector subset of sample first + s: keep j when
// u_j < lam_j / (lam_j + 1); sizes[s] = count, cols[s][0..count) ascending,
// the rest of the row -1.
__global__ void dpp_kernel(const double* lam, int d, uint64_t seed, uint64_t first, int n,
                           int32_t* cols, int32_t* sizes) {
#pragma clang fp contract(off)
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  int32_t* out = cols + (size_t)s * d;
  int c = 0;
  for (int j = 0; j < d; ++j) {
    const double u = uniform53(philox_stream(seed, first + (uint64_t)s, (uint32_t)j, kSelectStream));
    const double lj = lam[j];
    if (u < lj / (lj + 1.0)) out[c++] = j;
  }
  sizes[s] = c;
  for (int j = c; j < d; ++j) out[j] = -1;
}

__global__ void fill_rows_kernel(int32_t* x, double* logdet, int n, int N) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < (size_t)n * N) x[i] = -1;
  if (logdet && i < (size_t)n) logdet[i] = 0.0;
}

__global__ void gather_rows_kernel(const int32_t* src, int lds, const int32_t* pos, int n, int k,
                                   int32_t* dst) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)n * k) return;
  const size_t r = i / k, c = i % k;
  dst[i] = src[(size_t)pos[r] * lds + c];
}

__global__ void scatter_rows_kernel(const int32_t* xb, const double* ldb, const int32_t* pos,
                                    int n, int k, int32_t* x, int ldx, double* logdet) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)n * k) return;
  const size_t r = i / k, c = i % k;
  x[(size_t)pos[r] * ldx + c] = xb[i];
  if (logdet && ldb && c == 0) logdet[pos[r]] = ldb[r];
}

__global__ void stats_add_kernel(const int32_t* ctl, const unsigned long long* counters,
                                 unsigned long long* acc) {
  // size groups may run on several streams at once: integer atomics, so the
  // totals do not depend on their order
  if (threadIdx.x != 0) return;
  atomicOr(&acc[0], (unsigned long long)(uint32_t)ctl[1]);
  atomicAdd(&acc[1], counters[0]);
  atomicAdd(&acc[2], counters[1]);
}

__global__ void stats_store_kernel(const unsigned long long* acc, int32_t* ctl,
                                   unsigned long long* counters) {
  if (threadIdx.x != 0) return;
  ctl[1] = (int32_t)acc[0];
  counters[0] = acc[1];
  counters[1] = acc[2];
}

#define DPP_HIP(call)                                                       \
  do {                                                                      \
    hipError_t e_ = (call);                                                 \
    if (e_ != hipSuccess) {                                                 \
      set_error(FFS_ERR_HIP, hipGetErrorString(e_));                        \
      return FFS_ERR_HIP;                                                   \
    }                                                                       \
  } while (0)

}  // namespace

namespace ffsk {
static unsigned grid_for(size_t n) { return (unsigned)((n + 255) / 256); }
void launch_fill_rows(int32_t* x, double* logdet, int n, int N, hipStream_t st) {
  const size_t m = (size_t)n * N > (size_t)n ? (size_t)n * N : (size_t)n;
  hipLaunchKernelGGL(fill_rows_kernel, dim3(grid_for(m)), dim3(256), 0, st, x, logdet, n, N);
}
void launch_gather_rows(const int32_t* src, int lds, const int32_t* pos, int n, int k,
                        int32_t* dst, hipStream_t st) {
  hipLaunchKernelGGL(gather_rows_kernel, dim3(grid_for((size_t)n * k)), dim3(256), 0, st, src,
                     lds, pos, n, k, dst);
}
void launch_scatter_rows(const int32_t* xb, const double* ldb, const int32_t* pos, int n, int k,
                         int32_t* x, int ldx, double* logdet, hipStream_t st) {
  hipLaunchKernelGGL(scatter_rows_kernel, dim3(grid_for((size_t)n * k)), dim3(256), 0, st, xb,
                     ldb, pos, n, k, x, ldx, logdet);
}
void launch_stats_add(const int32_t* ctl, const unsigned long long* counters,
                      unsigned long long* acc, hipStream_t st) {
  hipLaunchKernelGGL(stats_add_kernel, dim3(1), dim3(64), 0, st, ctl, counters, acc);
}
void launch_stats_store(const unsigned long long* acc, int32_t* ctl,
                        unsigned long long* counters, hipStream_t st) {
  hipLaunchKernelGGL(stats_store_kernel, dim3(1), dim3(64), 0, st, acc, ctl, counters);
}
}  // namespace ffsk

extern "C" {

ffs_status ffs_dpp_eig(const double* B_dev, int64_t L, int64_t d, double* lambda_dev,
                       double* U_dev, double* W_dev, int32_t* sweeps_out, void* stream) {
  if (!B_dev || !lambda_dev || !U_dev)
    return (ffs_status)set_error(FFS_ERR_INVALID_ARG, "NULL B_dev, lambda_dev or U_dev");
  if (d < 1 || L < d)
    return (ffs_status)set_error(FFS_ERR_INVALID_ARG, "need 1 <= d <= L");
  if (d > kDppMaxD)
    return (ffs_status)set_error(FFS_ERR_UNSUPPORTED, "dual dimension d above 512");
  if (L > (int64_t)1 << 26)
    return (ffs_status)set_error(FFS_ERR_UNSUPPORTED, "L above 2^26");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int di = (int)d, Li = (int)L;
  const size_t mat = (size_t)d * d * sizeof(double);
  char* buf = nullptr;
  DPP_HIP(hipMallocAsync((void**)&buf, 4 * mat + 256, st));
  double* A = reinterpret_cast<double*>(buf);
  double* V = reinterpret_cast<double*>(buf + mat);
  double* W = W_dev ? W_dev : reinterpret_cast<double*>(buf + 2 * mat);
  double* A2 = reinterpret_cast<double*>(buf + 3 * mat);
  int* info = reinterpret_cast<int*>(buf + 4 * mat);
  const unsigned gd = (unsigned)((d + 31) / 32);
  hipLaunchKernelGGL(gram_kernel, dim3(gd, gd), dim3(256), 0, st, B_dev, Li, di, A);
  // Cyclic Jacobi, one launch per round (d - 1 or d per sweep) over the whole
  // chip; the host reads one flag per sweep and stops after a sweep that
  // rotated nothing.
  const int n = di + (di & 1), np = n / 2;
  const unsigned rblocks = (unsigned)((np * np + di * np + 255) / 256);
  hipLaunchKernelGGL(identity_kernel, dim3((unsigned)(((size_t)d * d + 255) / 256)), dim3(256), 0,
                     st, V, di);
  double* Ain = A;
  double* Aout = A2;
  int sweep = 0, still = 1;
  while (still && sweep < kMaxSweeps) {
    DPP_HIP(hipMemsetAsync(info, 0, sizeof(int), st));
    for (int r = 0; r < n - 1; ++r) {
      hipLaunchKernelGGL(jacobi_round_kernel, dim3(rblocks), dim3(256), 0, st, Ain, Aout, V, di, n,
                         r, 1e-14, info);
      double* tmp = Ain;
      Ain = Aout;
      Aout = tmp;
    }
    int flag = 0;
    DPP_HIP(hipMemcpyAsync(&flag, info, sizeof(int), hipMemcpyDeviceToHost, st));
    DPP_HIP(hipStreamSynchronize(st));
    ++sweep;
    still = flag;
  }
  hipLaunchKernelGGL(order_kernel, dim3((unsigned)((d + 255) / 256)), dim3(256), 0, st, Ain, V, di,
                     lambda_dev, W);
  std::vector<double> lam((size_t)d);
  DPP_HIP(hipMemcpyAsync(lam.data(), lambda_dev, d * sizeof(double), hipMemcpyDeviceToHost, st));
  DPP_HIP(hipStreamSynchronize(st));
  if (sweeps_out) *sweeps_out = sweep;
  ffs_status rc = FFS_OK;
  if (still) {
    rc = (ffs_status)set_error(FFS_ERR_NUMERICAL, "Jacobi did not converge in 60 sweeps");
  } else if (!(lam[0] > 1e-12 * lam[d - 1])) {
    rc = (ffs_status)set_error(FFS_ERR_NUMERICAL,
                               "B^T B is numerically singular (lambda_min <= 1e-12 lambda_max)");
  } else {
    hipLaunchKernelGGL(project_kernel, dim3((unsigned)((L + 31) / 32), gd), dim3(256), 0, st,
                       B_dev, W, lambda_dev, Li, di, U_dev);
  }
  DPP_HIP(hipFreeAsync(buf, st));
  DPP_HIP(hipGetLastError());
  DPP_HIP(hipStreamSynchronize(st));
  return rc;
}

ffs_status ffs_kdpp_subsets(const double* lambda_dev, int64_t d, int64_t k, uint64_t seed,
                            uint64_t first_sample, int64_t n, int32_t* cols_dev, void* stream) {
  if (!lambda_dev || (n > 0 && !cols_dev))
    return (ffs_status)set_error(FFS_ERR_INVALID_ARG, "NULL lambda_dev or cols_dev");
  if (d < 1 || k < 1 || k > d || n < 0)
    return (ffs_status)set_error(FFS_ERR_INVALID_ARG, "need 1 <= k <= d and n >= 0");
  if (d > 65536 || n > ((int64_t)1 << 31) - 1)
    return (ffs_status)set_error(FFS_ERR_UNSUPPORTED, "d or n too large");
  if (n == 0) return FFS_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const size_t tbytes = (size_t)(k + 1) * (d + 1) * sizeof(double);
  char* buf = nullptr;
  DPP_HIP(hipMallocAsync((void**)&buf, tbytes + 256, st));
  double* E = reinterpret_cast<double*>(buf);
  int* status = reinterpret_cast<int*>(buf + tbytes);
  DPP_HIP(hipMemsetAsync(status, 0, sizeof(int), st));
  hipLaunchKernelGGL(esp_kernel, dim3(1), dim3(64), 0, st, lambda_dev, (int)d, (int)k, E, status);
  int h = 0;
  DPP_HIP(hipMemcpyAsync(&h, status, sizeof(int), hipMemcpyDeviceToHost, st));
  DPP_HIP(hipStreamSynchronize(st));
  ffs_status rc = FFS_OK;
  if (h) {
    rc = (ffs_status)set_error(FFS_ERR_NUMERICAL,
                               "eigenvalues negative or e_k of the scaled eigenvalues out of range");
  } else {
    hipLaunchKernelGGL(kdpp_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, lambda_dev,
                       E, (int)d, (int)k, seed, first_sample, (int)n, cols_dev);
  }
  DPP_HIP(hipFreeAsync(buf, st));
  DPP_HIP(hipGetLastError());
  return rc;
}

ffs_status ffs_dpp_subsets(const double* lambda_dev, int64_t d, uint64_t seed,
                           uint64_t first_sample, int64_t n, int32_t* cols_dev,
                           int32_t* sizes_dev, void* stream) {
  if (!lambda_dev || (n > 0 && (!cols_dev || !sizes_dev)))
    return (ffs_status)set_error(FFS_ERR_INVALID_ARG, "NULL lambda_dev, cols_dev or sizes_dev");
  if (d < 1 || n < 0) return (ffs_status)set_error(FFS_ERR_INVALID_ARG, "need d >= 1 and n >= 0");
  if (d > 65536 || n > ((int64_t)1 << 31) - 1)
    return (ffs_status)set_error(FFS_ERR_UNSUPPORTED, "d or n too large");
  if (n == 0) return FFS_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(dpp_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, lambda_dev,
                     (int)d, seed, first_sample, (int)n, cols_dev, sizes_dev);
  DPP_HIP(hipGetLastError());
  return FFS_OK;
}

}  // extern "C"
