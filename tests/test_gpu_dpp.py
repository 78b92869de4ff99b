"""GPU parity of the DPP front end (applications section): the dual
eigendecomposition against the oracle's, the eigenvector selections bit for
bit against the oracle's on the same eigenvalues, and the whole pipeline
(features -> eigenvectors -> selection -> fermion sampling) against the
oracle's pipeline from the same features."""
import sys

import numpy as np
import pytest

from oracle import dpp, sampler
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


# eigenvalues: 1e-12 of the largest; eigenvectors: the float64 perturbation
# bound eps * lambda_max / gap stays far below 1e-8 for these spectra.
LAM_TOL = 1e-12
VEC_TOL = 1e-8


@pytest.mark.parametrize("L,d,scale", [(300, 40, 1.0), (2000, 64, 0.3), (20000, 256, 1.0)])
def test_dual_eig_matches_oracle(ffs, L, d, scale):
    import torch
    say("case dpp eig L=%d d=%d scale=%g" % (L, d, scale))
    B = workloads.dpp_features(L, d, seed=4) * scale
    lam, U, W, sweeps = ffs.ffs_dpp_eig(torch.from_numpy(B).cuda())
    lo, Uo, Wo = dpp.dual_eig(B)
    lam, U, W = lam.cpu().numpy(), U.cpu().numpy(), W.cpu().numpy()
    say("  sweeps", sweeps, "lambda range", lo[0], lo[-1])
    assert 0 < sweeps <= 30
    assert np.abs(lam - lo).max() <= LAM_TOL * lo[-1]
    assert np.abs(W - Wo).max() <= VEC_TOL
    assert np.abs(U - Uo).max() <= VEC_TOL
    assert np.abs(U.T @ U - np.eye(d)).max() <= 1e-10


@pytest.mark.parametrize("d,k", [(64, 1), (256, 10), (256, 50), (40, 40)])
def test_kdpp_subsets_bit_exact(ffs, d, k):
    import torch
    say("case kdpp selection d=%d k=%d" % (d, k))
    lo, _, _ = dpp.dual_eig(workloads.dpp_features(4 * d + 50, d, seed=9))
    n, seed, first = 96, 1234, 5000
    cols = ffs.ffs_kdpp_subsets(torch.from_numpy(lo).cuda(), k, seed, first, n).cpu().numpy()
    E = dpp.esp_table(lo, k)
    for s in range(n):
        assert list(cols[s]) == dpp.kdpp_select(lo, k, seed, first + s, E=E), s


@pytest.mark.parametrize("scale", [1.0, 0.02])
def test_dpp_subsets_bit_exact(ffs, scale):
    import torch
    d = 128
    say("case dpp selection d=%d scale=%g" % (d, scale))
    lo, _, _ = dpp.dual_eig(workloads.dpp_features(1000, d, seed=6) * scale)
    n, seed, first = 80, 99, 7
    cols, sizes = ffs.ffs_dpp_subsets(torch.from_numpy(lo).cuda(), seed, first, n)
    cols, sizes = cols.cpu().numpy(), sizes.cpu().numpy()
    say("  mean size", sizes.mean(), "expected", (lo / (lo + 1)).sum())
    for s in range(n):
        J = dpp.dpp_select(lo, seed, first + s)
        assert sizes[s] == len(J)
        assert list(cols[s, :len(J)]) == J
        assert np.all(cols[s, len(J):] == -1)


def test_dpp_pipeline_matches_oracle(ffs):
    import torch
    L, d, k, n = 1500, 48, 8, 40
    seed_sel, seed_smp = 21, 77
    say("case dpp pipeline L=%d d=%d k=%d n=%d" % (L, d, k, n))
    B = workloads.dpp_features(L, d, seed=12)
    lam, U, _, _ = ffs.ffs_dpp_eig(torch.from_numpy(B).cuda())
    cols = ffs.ffs_kdpp_subsets(lam, k, seed_sel, 0, n)
    plan = ffs.ffs_plan(U)
    x, _ = ffs.ffs_sample_subsets(plan, cols, seed_smp, 300)
    torch.cuda.synchronize()
    st = ffs.ffs_check(plan)
    assert st["device_status"] == 0
    X, C = x.cpu().numpy(), cols.cpu().numpy()
    lo, Uo, _ = dpp.dual_eig(B)
    E = dpp.esp_table(lo, k)
    tie = 0
    for s in range(n):
        J = dpp.kdpp_select(lo, k, seed_sel, s, E=E)
        assert list(C[s]) == J, s
        r = sampler.sample_one(Uo[:, J], seed_smp, 300 + s)
        if not np.array_equal(X[s], r["x"]):
            j = int(np.argmax(X[s] != np.array(r["x"])))
            assert r["margin"][j] < 1e-9
            tie += 1
    say("  ties", tie)
    assert tie <= 1


def test_dpp_errors(ffs):
    import torch
    from paper_2109_07358_amd.ffs import FFSError
    B = torch.zeros((10, 20), dtype=torch.float64, device="cuda")
    with pytest.raises(FFSError):          # d > L
        ffs.ffs_dpp_eig(B)
    with pytest.raises(FFSError):          # rank-deficient features
        Bs = workloads.dpp_features(50, 6, seed=3)
        Bs[:, 5] = Bs[:, 4]
        ffs.ffs_dpp_eig(torch.from_numpy(Bs).cuda())
    lam = torch.tensor([1.0, 2.0, 3.0], dtype=torch.float64, device="cuda")
    with pytest.raises(FFSError):          # k > d
        ffs.ffs_kdpp_subsets(lam, 4, 1, 0, 5)
    with pytest.raises(FFSError):          # negative eigenvalue
        ffs.ffs_kdpp_subsets(torch.tensor([1.0, -2.0, 3.0], dtype=torch.float64,
                                          device="cuda"), 2, 1, 0, 5)


@pytest.mark.parametrize("bulk", ["fp32", "split_bf16"])
def test_dpp_variable_size_pipeline(ffs, bulk):
    # the paper's rule: eigenvector j kept with probability lambda_j/(lambda_j+1),
    # then each sample draws as many items as it kept eigenvectors
    import torch
    L, d, n = 1500, 48, 60
    seed_sel, seed_smp, first = 5, 41, 900
    say("case dpp variable sizes L=%d d=%d n=%d %s" % (L, d, n, bulk))
    B = workloads.dpp_features(L, d, seed=13) * 0.09
    lam, U, _, _ = ffs.ffs_dpp_eig(torch.from_numpy(B).cuda())
    cols, sizes = ffs.ffs_dpp_subsets(lam, seed_sel, first, n)
    plan = ffs.ffs_plan(U, bulk=bulk)
    x, ld = ffs.ffs_sample_dpp(plan, cols, sizes, seed_smp, first, logdet=True)
    torch.cuda.synchronize()
    st = ffs.ffs_check(plan)
    X, SZ, LD = x.cpu().numpy(), sizes.cpu().numpy(), ld.cpu().numpy()
    say("  sizes", np.bincount(SZ), "stats", st)
    assert st["device_status"] == 0 and st["draws"] == int(SZ.sum())
    lo, Uo, _ = dpp.dual_eig(B)
    tie = 0
    for s in range(n):
        J = dpp.dpp_select(lo, seed_sel, first + s)
        assert SZ[s] == len(J)
        assert np.all(X[s, len(J):] == -1)
        if not J:
            assert LD[s] == 0.0
            continue
        r = sampler.sample_one(Uo[:, J], seed_smp, first + s)
        if not np.array_equal(X[s, :len(J)], r["x"]):
            j = int(np.argmax(X[s, :len(J)] != np.array(r["x"])))
            assert r["margin"][j] < 1e-9
            tie += 1
            continue
        _, l = np.linalg.slogdet(Uo[np.array(r["x"])][:, J])
        assert abs(LD[s] - 2 * l) < 1e-8 * max(1.0, abs(l))
    say("  ties", tie)
    assert tie <= 1
