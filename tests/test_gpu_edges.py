"""GPU edge cases through the C ABI: degenerate shapes, empty calls, the
largest supported sizes and the working-memory budget."""
import sys

import numpy as np
import pytest

from oracle import sampler
from paper_2109_07358_amd import workloads

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ffs():
    import torch
    from paper_2109_07358_amd import ffs as f
    f.load()
    torch.cuda.set_device(0)
    return f


def _rows_match(U, X, seed, first, idx, n_keep=None):
    for i in idx:
        r = sampler.sample_one(U, seed, first + i, n_keep)
        if not np.array_equal(X[i][: len(r["x"])], r["x"]):
            k = int(np.argmax(X[i][: len(r["x"])] != np.array(r["x"])))
            assert r["margin"][k] < 1e-9, (i, k)


@pytest.mark.parametrize("path", ["batched", "plain"])
def test_single_particle(ffs, path):
    """N = 1: x is drawn from |U[x, 0]|^2 directly."""
    import torch
    U = workloads.gaussian_qr(333, 1, 3)
    plan = ffs.ffs_plan(U, path=path)
    x, ld = ffs.ffs_sample(plan, 5, 0, 200, logdet=True)
    torch.cuda.synchronize()
    X, LD = x.cpu().numpy(), ld.cpu().numpy()
    _rows_match(U, X, 5, 0, range(0, 200, 7))
    assert np.allclose(LD, np.log(U[X[:, 0], 0] ** 2), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("cplx", [False, True])
def test_full_filling_l_equals_n(ffs, cplx):
    """L = N: every site is drawn, |det U| = 1, so x is a permutation and
    the log-determinant is 0."""
    import torch
    U = workloads.gaussian_qr(40, 40, 6, complex_=cplx)
    plan = ffs.ffs_plan(U)
    x, ld = ffs.ffs_sample(plan, 2, 0, 130, logdet=True)
    torch.cuda.synchronize()
    X = x.cpu().numpy()
    assert all(sorted(r) == list(range(40)) for r in X)
    assert np.max(np.abs(ld.cpu().numpy())) < 1e-9
    _rows_match(U, X, 2, 0, [0, 77, 129])


def test_empty_and_trivial_calls(ffs):
    import torch
    U = workloads.gaussian_qr(100, 10, 2)
    plan = ffs.ffs_plan(U)
    x = torch.full((4, 10), -7, dtype=torch.int32, device="cuda")
    ffs.ffs_sample(plan, 1, 0, 0, x_out=x)          # n = 0: no-op
    ffs.ffs_marginal(plan, 0, 1, 0, 4, x_out=x)      # n_keep = 0: no-op
    torch.cuda.synchronize()
    assert (x.cpu().numpy() == -7).all()
    one, _ = ffs.ffs_sample(plan, 9, 41, 1)          # a single sample
    torch.cuda.synchronize()
    _rows_match(U, one.cpu().numpy(), 9, 41, [0])
    m1 = ffs.ffs_marginal(plan, 1, 9, 41, 1)         # first particle only
    torch.cuda.synchronize()
    assert m1.cpu().numpy()[0, 0] == one.cpu().numpy()[0, 0]


def test_largest_sites(ffs):
    """L = 65536 (the largest supported), N = 16, sampled rows vs the oracle."""
    import torch
    say("case L=65536 N=16 S=300")
    U = workloads.gaussian_qr(65536, 16, 7)
    plan = ffs.ffs_plan(U)
    x, _ = ffs.ffs_sample(plan, 3, 0, 300)
    torch.cuda.synchronize()
    X = x.cpu().numpy()
    assert X.max() < 65536 and all(len(set(r)) == 16 for r in X)
    _rows_match(U, X, 3, 0, [0, 150, 299])


def test_largest_particles_sampled(ffs):
    """N = 1024 (the largest supported) at L = 4096: oracle marginal on a
    prefix, log-determinant identity on whole samples."""
    import torch
    say("case L=4096 N=1024 S=64")
    U = workloads.gaussian_qr(4096, 1024, 8)
    plan = ffs.ffs_plan(U)
    x, ld = ffs.ffs_sample(plan, 4, 0, 64, logdet=True)
    torch.cuda.synchronize()
    X, LD = x.cpu().numpy(), ld.cpu().numpy()
    assert all(len(set(r)) == 1024 for r in X)
    for i in (0, 63):
        _, l = np.linalg.slogdet(U[X[i]])
        assert abs(LD[i] - 2 * l) < 1e-7 * max(1.0, abs(l))
    _rows_match(U, X, 4, 0, [0, 63], n_keep=40)


def test_hbm_budget_chunks_the_batch(ffs):
    """A working-memory budget below one full batch splits the call into
    chunks; the result is unchanged."""
    import torch
    U = workloads.gaussian_qr(1000, 64, 9)
    full = ffs.ffs_plan(U)
    small = ffs.ffs_plan(U, hbm_budget=24 << 20)
    a, _ = ffs.ffs_sample(full, 6, 0, 1000)
    b, _ = ffs.ffs_sample(small, 6, 0, 1000)
    torch.cuda.synchronize()
    assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())


@pytest.mark.parametrize("n", [257, 383])
def test_lopsided_half_batches(ffs, n):
    """Batches just over the split threshold run as a 256-sample half and a
    1- or 127-sample half on two streams: each sample equals the same sample
    drawn in a single-stream call, and the last rows match the oracle."""
    import torch
    say("case lopsided halves n=%d" % n)
    U = workloads.gaussian_qr(700, 33, 10)
    two = ffs.ffs_plan(U)
    one = ffs.ffs_plan(U, overlap=False)
    a, la = ffs.ffs_sample(two, 8, 1000, n, logdet=True)
    b, lb = ffs.ffs_sample(one, 8, 1000, n, logdet=True)
    torch.cuda.synchronize()
    A = a.cpu().numpy()
    assert np.array_equal(A, b.cpu().numpy())
    assert np.array_equal(la.cpu().numpy(), lb.cpu().numpy())
    assert all(len(set(r)) == 33 for r in A)
    _rows_match(U, A, 8, 1000, [0, 255, 256, n - 1])
