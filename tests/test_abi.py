"""CPU-side checks of the C ABI: the library loads, exports every symbol the
header declares, and its host-side logic (validation, Philox) is right.
No device compute is called here."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import philox
from paper_2109_07358_amd import ffs, workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ffs.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ffs_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = ffs.load()
    syms = declared_symbols()
    assert len(syms) >= 10
    for s in syms:
        assert hasattr(lib, s), s
    assert set(syms) == set(ffs.EXPORTS)


def test_host_philox_matches_oracle():
    rng = np.random.default_rng(0)
    for _ in range(50):
        seed = int(rng.integers(0, 2 ** 63)) * 2 + int(rng.integers(0, 2))
        s = int(rng.integers(0, 2 ** 40))
        t = int(rng.integers(0, 1024))
        assert ffs.ffs_philox_words(seed, s, t) == philox.step_words(seed, s, t)


def test_default_options():
    o = ffs.ffs_default_options()
    assert o.bulk == ffs.BULK["fp32"] and o.path == ffs.PATH["batched"]
    assert o.ortho_tol == 1e-10 and o.guard_delta == -1.0 and o.guard_scale == -1.0
    assert o.max_batch == 4096 and o.hbm_budget == 0


def _plan_status(U, L=None, N=None, ldu=None, dtype=0, opt=None):
    lib = ffs.load()
    h = ctypes.c_void_p()
    U = np.ascontiguousarray(U)
    L = U.shape[0] if L is None else L
    N = U.shape[1] if N is None else N
    ldu = N if ldu is None else ldu
    o = ffs.ffs_default_options() if opt is None else opt
    st = lib.ffs_plan(ctypes.byref(h), U.ctypes.data, L, N, ldu, dtype,
                      ctypes.byref(o))
    return st, h


def test_plan_rejects_bad_shapes_before_touching_the_device():
    U = workloads.gaussian_qr(16, 4, 0)
    assert _plan_status(U, L=3, N=4)[0] == -1          # N > L
    assert _plan_status(U, N=0)[0] == -1               # N < 1
    assert _plan_status(U, ldu=2)[0] == -1             # ldu < N
    assert _plan_status(U, dtype=7)[0] == -1           # dtype
    assert _plan_status(np.zeros((2000, 1100)))[0] == -6  # N > 1024
    o = ffs.ffs_default_options()
    o.bulk = 0  # float64 bulk on the batched path
    assert _plan_status(U, opt=o)[0] == -6
    assert "float64 bulk" in ffs.ffs_last_error()


def test_plan_rejects_non_orthonormal_and_non_finite():
    U = workloads.gaussian_qr(64, 8, 1).copy()
    U[3, 2] += 1e-6
    st, _ = _plan_status(U)
    assert st == -2 and "U^H U" in ffs.ffs_last_error()
    U[3, 2] = np.nan
    assert _plan_status(U)[0] == -5
    # randomised check path (L*N^2 > 2^28)
    V = workloads.gaussian_qr(20000, 128, 2).copy()
    V[100, 5] += 1e-6   # |U^T U - 1| ~ 1e-8 on row/column 5
    assert _plan_status(V)[0] == -2


def test_plan_rejects_non_orthonormal_complex():
    U = workloads.gaussian_qr(32, 4, 3, complex_=True).copy()
    U[0, 0] += 1e-7j
    h = ctypes.c_void_p()
    o = ffs.ffs_default_options()
    st = ffs.load().ffs_plan(ctypes.byref(h), U.ctypes.data, 32, 4, 4, 1,
                             ctypes.byref(o))
    assert st == -2


def test_null_arguments():
    lib = ffs.load()
    assert lib.ffs_plan(None, None, 4, 2, 2, 0, None) == -1
    assert lib.ffs_sample(None, 0, 0, 1, None, None, None) == -1
    assert lib.ffs_sample_noalloc(None, 0, 0, 1, None, None, None) == -1
    assert lib.ffs_check(None, None) == -1
    assert lib.ffs_destroy(None) == 0


def test_server_default_options():
    o = ffs.ServerOptions()
    ffs.load().ffs_server_default_options(ctypes.byref(o))
    assert o.mode == 0 and o.slots == 4 and o.hbm_budget == 0
    assert o.capacity == 128 and o.ticks == 8


def test_server_null_arguments():
    lib = ffs.load()
    info = ffs.RequestInfo()
    assert lib.ffs_server_create(None, None) == -1
    assert lib.ffs_server_poll(None, 1, 0, ctypes.byref(info)) == -1
    assert lib.ffs_server_destroy(None) == -1
    t = ctypes.c_uint64()
    assert lib.ffs_server_submit(None, None, 1, 0, 0, 1, None, None, ctypes.byref(t)) == -1


def test_group_argument_checks_before_the_device():
    lib = ffs.load()
    arr = (ffs.Instance * 1)()
    assert lib.ffs_sample_group(arr, 0, 0, None, None) == 0
    assert lib.ffs_sample_group(None, 2, 0, None, None) == -1
    assert lib.ffs_sample_group(arr, 1, 8, None, None) == -1


def test_tuning_hooks_reject_bad_arguments():
    lib = ffs.load()
    assert lib.ffs_autotune(None, 10, 0, None) == -1
    assert lib.ffs_set_tile(None, 10, 128, 128, 0) == -1


def test_widened_entry_points_reject_bad_arguments():
    # every check below returns before any device call
    lib = ffs.load()
    INVALID, UNSUP = -1, -6
    vp = ctypes.c_void_p(0x1000)   # never dereferenced: the calls fail first
    # dual eigendecomposition: NULL pointers, d > L, d above the Jacobi limit
    assert lib.ffs_dpp_eig(None, 10, 4, vp, vp, None, None, None) == INVALID
    assert lib.ffs_dpp_eig(vp, 3, 4, vp, vp, None, None, None) == INVALID
    assert lib.ffs_dpp_eig(vp, 2000, 600, vp, vp, None, None, None) == UNSUP
    # selections: k outside [1, d], negative n, NULL outputs
    assert lib.ffs_kdpp_subsets(vp, 8, 9, 1, 0, 4, vp, None) == INVALID
    assert lib.ffs_kdpp_subsets(vp, 8, 0, 1, 0, 4, vp, None) == INVALID
    assert lib.ffs_kdpp_subsets(vp, 8, 2, 1, 0, -1, vp, None) == INVALID
    assert lib.ffs_kdpp_subsets(vp, 8, 2, 1, 0, 0, vp, None) == 0     # n = 0: no-op
    assert lib.ffs_dpp_subsets(vp, 8, 1, 0, 4, None, vp, None) == INVALID
    assert lib.ffs_dpp_subsets(vp, 0, 1, 0, 4, vp, vp, None) == INVALID
    # Jastrow estimate: sizes, L limit, non-finite V
    assert lib.ffs_jastrow_estimate(vp, 0, None, 0, 4, 10, 1.0, None, None, vp, vp, vp, None) == INVALID
    assert lib.ffs_jastrow_estimate(vp, 2, None, 3, 4, 10, 1.0, None, None, vp, vp, vp, None) == INVALID
    assert lib.ffs_jastrow_estimate(vp, 2, None, 0, 4, 70000, 1.0, None, None, vp, vp, vp, None) == UNSUP
    assert lib.ffs_jastrow_estimate(vp, 2, None, 0, 4, 10, float("nan"), None, None, vp, vp, vp,
                                    None) == INVALID
    # plan from device memory: argument errors before any copy
    h = ctypes.c_void_p()
    o = ffs.ffs_default_options()
    assert lib.ffs_plan_device(ctypes.byref(h), None, 10, 2, 2, 0, ctypes.byref(o)) == INVALID
    assert lib.ffs_plan_device(ctypes.byref(h), vp, 2, 3, 3, 0, ctypes.byref(o)) == INVALID
    assert lib.ffs_plan_device(ctypes.byref(h), vp, 10, 2, 2, 7, ctypes.byref(o)) == INVALID
    # calls on a NULL plan
    acc = ctypes.c_int64()
    assert lib.ffs_sample_mh(None, 4, 0, 1, 0, 8, vp, None, ctypes.byref(acc), None) == INVALID
    assert lib.ffs_sample_dpp(None, vp, vp, 1, 0, 8, vp, None, None) == INVALID
    assert lib.ffs_set_timing_classes(None, 1) == INVALID
    assert lib.ffs_set_timing_stride(None, 2) == INVALID
