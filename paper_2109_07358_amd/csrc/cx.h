// Real / complex float64 scalar operations used by the factor and repair
// kernels.  Complex numbers are double2 (x = re, y = im).  All products are
// bilinear (no implicit conjugation): the normal vector h of Eq. (3) is
// read as u_{x_i}^T h = 0, which keeps |u^T h|^2 proportional to |det|^2.
#pragma once

#include <hip/hip_runtime.h>

namespace ffsk {

template <bool C>
struct Cx;

template <>
struct Cx<false> {
  using T = double;
  __device__ static T zero() { return 0.0; }
  __device__ static T one() { return 1.0; }
  __device__ static T add(T a, T b) { return a + b; }
  __device__ static T sub(T a, T b) { return a - b; }
  __device__ static T mul(T a, T b) { return a * b; }
  __device__ static T neg(T a) { return -a; }
  // c + a*b
  __device__ static T fma(T a, T b, T c) { return __fma_rn(a, b, c); }
  // c - a*b
  __device__ static T fnma(T a, T b, T c) { return __fma_rn(-a, b, c); }
  __device__ static T inv(T a) { return 1.0 / a; }
  __device__ static double abs2(T a) { return a * a; }
  __device__ static bool finite(T a) { return isfinite(a); }
  __device__ static T shfl_xor(T a, int m) { return __shfl_xor(a, m, 64); }
  __device__ static T bcast(T a, int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(a), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(a), lane);
    return __hiloint2double(hi, lo);
  }
  __device__ static double re(T a) { return a; }
  __device__ static double im(T) { return 0.0; }
};

template <>
struct Cx<true> {
  using T = double2;
  __device__ static T zero() { return make_double2(0.0, 0.0); }
  __device__ static T one() { return make_double2(1.0, 0.0); }
  __device__ static T add(T a, T b) { return make_double2(a.x + b.x, a.y + b.y); }
  __device__ static T sub(T a, T b) { return make_double2(a.x - b.x, a.y - b.y); }
  __device__ static T mul(T a, T b) {
    return make_double2(__fma_rn(a.x, b.x, -a.y * b.y),
                        __fma_rn(a.x, b.y, a.y * b.x));
  }
  __device__ static T neg(T a) { return make_double2(-a.x, -a.y); }
  __device__ static T fma(T a, T b, T c) {
    return make_double2(__fma_rn(a.x, b.x, __fma_rn(-a.y, b.y, c.x)),
                        __fma_rn(a.x, b.y, __fma_rn(a.y, b.x, c.y)));
  }
  __device__ static T fnma(T a, T b, T c) {
    return make_double2(__fma_rn(-a.x, b.x, __fma_rn(a.y, b.y, c.x)),
                        __fma_rn(-a.x, b.y, __fma_rn(-a.y, b.x, c.y)));
  }
  __device__ static T inv(T a) {
    const double d = a.x * a.x + a.y * a.y;
    return make_double2(a.x / d, -a.y / d);
  }
  __device__ static double abs2(T a) { return a.x * a.x + a.y * a.y; }
  __device__ static bool finite(T a) { return isfinite(a.x) && isfinite(a.y); }
  __device__ static T shfl_xor(T a, int m) {
    return make_double2(__shfl_xor(a.x, m, 64), __shfl_xor(a.y, m, 64));
  }
  __device__ static T bcast(T a, int lane) {
    return make_double2(Cx<false>::bcast(a.x, lane), Cx<false>::bcast(a.y, lane));
  }
  __device__ static double re(T a) { return a.x; }
  __device__ static double im(T a) { return a.y; }
};

// Orders LDS traffic between the lanes of one wavefront.  A wavefront's LDS
// instructions complete in issue order, so a compiler-level barrier with a
// wavefront-scope fence is enough; no s_barrier is involved, which lets one
// wavefront of a larger workgroup run alone (or exit early) safely.
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Wave-wide sum (64 lanes), fixed butterfly order: every lane gets the same
// bits.
template <bool C>
__device__ inline typename Cx<C>::T wave_sum(typename Cx<C>::T v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v = Cx<C>::add(v, Cx<C>::shfl_xor(v, m));
  return v;
}

}  // namespace ffsk
