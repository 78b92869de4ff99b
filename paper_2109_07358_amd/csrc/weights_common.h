// Pieces shared by the float32 (k_weights.hip) and split-BF16
// (k_weights_bf16.hip) all-site weight contractions: the accumulator type,
// the fused epilogue, the launch-span stamps and the launch helper.
#pragma once
#include <hip/hip_ext.h>

#include "args.h"
#include "ffs_internal.h"

namespace ffsk {

typedef float floatx16 __attribute__((ext_vector_type(16)));

namespace wk {

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

// The real epilogue of a wavefront's 32 x 32 tile (sites sb..sb+31,
// samples smp0w..smp0w+31) with the weights staged through st (32 x 32
// floats of LDS, this wavefront's own; the 16-byte slot of sites 4k..4k+3
// of sample s at slot k ^ (s % 8), so that the 8-lane write phases and
// 16-lane read phases are conflict-free) and written back as whole 128-byte
// sample lines with non-temporal stores: 8 lanes per sample, 8 samples per
// instruction.  Same values and block sums as epilogue<false>.
__device__ inline void epilogue_lines(const WArgs& g, int nblk, int sb, int smp0w, int li, int kh,
                                      floatx16 acc, float* st) {
  const int smp = smp0w + li;
  const int blk = sb >> 5;
  const uint32_t occw = g.occ[(size_t)smp * nblk + blk];
  double part = 0.0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    float w4[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int r = 4 * q + c;
      const int row = 8 * q + 4 * kh + c;
      const float v = acc[r] * acc[r];
      w4[c] = ((occw >> row) & 1u) ? 0.0f : v;
      part += (double)w4[c];
    }
    const int slot = (2 * q + kh) ^ (li & 7);
    *reinterpret_cast<float4*>(st + li * 32 + 4 * slot) = make_float4(w4[0], w4[1], w4[2], w4[3]);
  }
  const double other = __shfl_xor(part, 32, 64);
  const double tot = (kh == 0) ? part + other : other + part;
  if (kh == 0) g.bsum[(size_t)smp * nblk + blk] = tot;
  const int lane = threadIdx.x & 63;
  typedef float f4 __attribute__((ext_vector_type(4)));
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int s = 8 * i + (lane >> 3), p = lane & 7;
    const f4 v = *reinterpret_cast<const f4*>(st + s * 32 + 4 * (p ^ (s & 7)));
    __builtin_nontemporal_store(v, reinterpret_cast<f4*>(g.wh + (size_t)(smp0w + s) * g.L_pad + sb + 4 * p));
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

// 256-thread launch; with events, stamped by the dispatch itself.
template <typename K, typename... A>
inline void launch256(K kernel, dim3 grid, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1, A... args) {
  if (ev0)
    hipExtLaunchKernelGGL(kernel, grid, dim3(256), 0, st, ev0, ev1, 0, args...);
  else
    hipLaunchKernelGGL(kernel, grid, dim3(256), 0, st, args...);
}

}  // namespace wk
}  // namespace ffsk
