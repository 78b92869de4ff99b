// Wavefront-level helpers shared by the float64 conditioning updates of the
// batched path (factor_blk.h) and the plain path (factor_wg.h).
#pragma once

#include "cx.h"
#include "ffs_internal.h"

namespace ffsk {

// Reduce-scatter of TW per-lane values over 64 lanes: on return lane l holds
// the full 64-lane sum of value number col(l) = l * TW / 64.  Fixed butterfly
// order (deterministic).
template <bool C, int TW>
__device__ inline typename Cx<C>::T reduce_scatter(typename Cx<C>::T (&a)[TW],
                                                   int lane) {
  using X = Cx<C>;
  int n = TW;
#pragma unroll
  for (int M = 32; M >= 1; M >>= 1) {
    if (n > 1) {
      const bool up = (lane & M) != 0;
      const int h = n >> 1;
#pragma unroll
      for (int i = 0; i < TW / 2; ++i) {
        if (i < h) {
          const typename X::T lo = a[i], hi = a[i + h];
          const typename X::T send = up ? lo : hi;
          const typename X::T keep = up ? hi : lo;
          a[i] = X::add(keep, X::shfl_xor(send, M));
        }
      }
      n = h;
    } else {
      a[0] = X::add(a[0], X::shfl_xor(a[0], M));
    }
  }
  return a[0];
}

}  // namespace ffsk
