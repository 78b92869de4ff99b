"""MI355X-native fast fermion sampling (FFS).

The sampler draws configurations x with probability |det U[x,:]|^2 / N! for
an L x N matrix U with orthonormal columns.  The compute path is a C-ABI
shared library of hand-written HIP kernels for gfx950 (csrc/, declared in
include/ffs.h); `ffs` is a thin ctypes binding over it.  Importing this
package loads nothing; the library is loaded on first use and its absence
is an error (there is no CPU fallback).
"""
__all__ = ["ffs", "workloads"]
