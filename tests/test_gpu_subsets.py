"""GPU parity of per-sample column subsets (the projection stage of DPP
sampling): sample s equals the oracle run on U[:, J_s] with the same seed
and sample index."""
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


def _subsets(n, d, k, seed):
    rng = np.random.default_rng(seed)
    return np.stack([rng.permutation(d)[:k] for _ in range(n)]).astype(np.int32)


@pytest.mark.parametrize("bulk,cplx", [("fp32", False), ("fp32", True), ("split_bf16", False)])
def test_subsets_match_oracle(ffs, bulk, cplx):
    import torch
    L, d, k, n = 700, 64, 13, 150
    say("case column subsets L=%d d=%d k=%d n=%d %s complex %s" % (L, d, k, n, bulk, cplx))
    V = workloads.gaussian_qr(L, d, 31, complex_=cplx)
    plan = ffs.ffs_plan(V, bulk=bulk)
    J = _subsets(n, d, k, 5)
    cols = torch.from_numpy(J).cuda()
    x, ld = ffs.ffs_sample_subsets(plan, cols, 77, 1000, logdet=True)
    torch.cuda.synchronize()
    st = ffs.ffs_check(plan)
    X, LD = x.cpu().numpy(), ld.cpu().numpy()
    say("  stats", st)
    assert st["device_status"] == 0 and st["draws"] == n * k
    eq = tie = 0
    for i in range(0, n, 3):
        U = V[:, J[i]]
        r = sampler.sample_one(U, 77, 1000 + i)
        if np.array_equal(X[i], r["x"]):
            eq += 1
        else:
            j = int(np.argmax(X[i] != np.array(r["x"])))
            assert r["margin"][j] < 1e-9
            tie += 1
        _, l = np.linalg.slogdet(U[X[i]])
        assert abs(LD[i] - 2 * l) < 1e-8 * max(1.0, abs(l))
    say("  equal", eq, "ties", tie)
    assert tie <= 1


def test_subsets_equal_plan_of_the_columns(ffs):
    """Same seed and sample index: the subset run equals ffs_sample on a plan
    built from U[:, J] (one J shared by all samples)."""
    import torch
    V = workloads.gaussian_qr(500, 48, 33)
    J = np.array([3, 40, 7, 22, 15, 9, 31, 0, 47, 12], dtype=np.int32)
    n = 200
    cols = torch.from_numpy(np.tile(J, (n, 1))).cuda()
    x, _ = ffs.ffs_sample_subsets(ffs.ffs_plan(V), cols, 5, 0)
    y, _ = ffs.ffs_sample(ffs.ffs_plan(np.ascontiguousarray(V[:, J])), 5, 0, n)
    torch.cuda.synchronize()
    assert np.array_equal(x.cpu().numpy(), y.cpu().numpy())


def test_subsets_report_bad_columns(ffs):
    import torch
    from paper_2109_07358_amd.ffs import FFSError
    V = workloads.gaussian_qr(300, 32, 34)
    plan = ffs.ffs_plan(V)
    J = np.array([[1, 2, 2], [0, 5, 31]], dtype=np.int32)  # a repeat in row 0
    ffs.ffs_sample_subsets(plan, torch.from_numpy(J).cuda(), 1, 0)
    torch.cuda.synchronize()
    with pytest.raises(FFSError):
        ffs.ffs_check(plan)
