"""GPU parity of the Slater-Jastrow reweighting (SI S-5) against the oracle:
log-weights, reweighted densities and double occupancy on seeded synthetic
configurations (several site tiles and sample groups, empty slots, spinless),
and on configurations drawn by the sampler for both spins."""
import sys

import numpy as np
import pytest

from oracle import jastrow, sampler
from paper_2109_07358_amd import workloads

pytestmark = pytest.mark.gpu

TOL = 1e-12   # float64 sums in a different order: relative to the scale of each quantity


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


def _check(ffs, xu, xd, L, V, vmat=None, extra=None):
    import torch
    c = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda() if a is not None else None
    lw, dens, summ = ffs.ffs_jastrow_estimate(c(xu), c(xd), L, V, vmat=c(vmat), extra_logw=c(extra))
    lo, do, so = jastrow.estimate(xu, xd, L, V, vmat=vmat, extra=extra)
    lw, dens = lw.cpu().numpy(), dens.cpu().numpy()
    scale = max(1.0, np.abs(lo).max())
    assert np.abs(lw - lo).max() <= TOL * scale
    assert np.abs(dens - do).max() <= TOL * max(1.0, np.abs(do).max())
    got = [summ[k] for k in ffs.JASTROW_SUMMARY]
    for g, o in zip(got, so):
        assert abs(g - o) <= 1e-11 * max(1.0, abs(o)), (got, so)
    return summ


@pytest.mark.parametrize("L,ku,kd,n,V,use_v,empty", [
    (300, 20, 17, 700, 0.9, True, 0.1),
    (5000, 64, 64, 1000, 2.0, False, 0.0),
    (2500, 40, 0, 600, 0.0, True, 0.05),
    (300, 30, 0, 200, 0.5, True, 0.0),
])
def test_jastrow_matches_oracle(ffs, L, ku, kd, n, V, use_v, empty):
    say("case jastrow L=%d ku=%d kd=%d n=%d V=%g vmat=%s" % (L, ku, kd, n, V, use_v))
    xu = workloads.random_configs(n, ku, L, 1, empty)
    xd = workloads.random_configs(n, kd, L, 2, empty) if kd else None
    rng = np.random.default_rng(3)
    vmat = None
    if use_v:
        a = rng.standard_normal((L, L)) * 0.01
        vmat = (a + a.T) / 2
    extra = rng.standard_normal(n) if use_v else None
    summ = _check(ffs, xu, xd, L, V, vmat, extra)
    say("  summary", summ)


def test_jastrow_pair_product_in_chunks(ffs):
    # L <= 16 (ku + kd) takes the pair term as a product on the FP64 matrix
    # cores, in chunks of samples whose counts fit 256 MB: 16128 rows at
    # L = 2048, so 16500 samples make two chunks.  Log-weights are per
    # sample: rows from both chunks and around the boundary against the
    # oracle (whose pair loop is too slow for all rows), and the unweighted
    # double occupancy of the whole run against the oracle's D
    import torch
    L, ku, kd, n, V = 2048, 64, 64, 16500, 0.7
    say("case jastrow pair product L=%d ku=%d kd=%d n=%d (two chunks)" % (L, ku, kd, n))
    xu = workloads.random_configs(n, ku, L, 5, 0.05)
    xd = workloads.random_configs(n, kd, L, 6, 0.05)
    rng = np.random.default_rng(7)
    a = rng.standard_normal((L, L)) * 0.01
    vmat = (a + a.T) / 2
    c = lambda z: torch.from_numpy(np.ascontiguousarray(z)).cuda()
    lw, dens, summ = ffs.ffs_jastrow_estimate(c(xu), c(xd), L, V, vmat=c(vmat))
    lw = lw.cpu().numpy()
    rows = np.r_[0:40, 16090:16170, 16460:16500]
    lo, _ = jastrow.log_weights(xu[rows], xd[rows], V, vmat)
    assert np.abs(lw[rows] - lo).max() <= TOL * max(1.0, np.abs(lo).max())
    _, D = jastrow.log_weights(xu, xd, V)
    assert abs(summ["D_0"] - D.mean()) <= 1e-12 * max(1.0, D.mean())


def test_jastrow_on_sampled_configurations(ffs):
    import torch
    L, N, n, V = 64, 8, 200, 1.5
    say("case jastrow on sampled configurations L=%d N=%d n=%d" % (L, N, n))
    U = workloads.gaussian_qr(L, N, 17)
    plan = ffs.ffs_plan(U)
    xu, _ = ffs.ffs_sample(plan, 101, 0, n)
    xd, _ = ffs.ffs_sample(plan, 202, 0, n)
    torch.cuda.synchronize()
    ou = np.array([sampler.sample_one(U, 101, s)["x"] for s in range(n)], dtype=np.int32)
    od = np.array([sampler.sample_one(U, 202, s)["x"] for s in range(n)], dtype=np.int32)
    assert np.array_equal(xu.cpu().numpy(), ou) and np.array_equal(xd.cpu().numpy(), od)
    lw, dens, summ = ffs.ffs_jastrow_estimate(xu, xd, L, V)
    lo, do, so = jastrow.estimate(ou, od, L, V)
    assert np.abs(lw.cpu().numpy() - lo).max() <= TOL * max(1.0, np.abs(lo).max())
    assert np.abs(dens.cpu().numpy() - do).max() <= TOL
    assert abs(summ["D_J"] - so[0]) <= 1e-11 and summ["D_J"] < summ["D_0"]


def test_jastrow_rejects_bad_sites(ffs):
    import torch
    from paper_2109_07358_amd.ffs import FFSError
    x = torch.tensor([[0, 5, 9]], dtype=torch.int32, device="cuda")
    with pytest.raises(FFSError):
        ffs.ffs_jastrow_estimate(x, None, 8, 1.0)
