"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Drawn sites are compared element by element on the same Philox stream.  The
bar: identical configurations, except where the oracle's own float64 draw
sits within 1e-9 (relative) of a CDF boundary -- a tie that float64 rounding
order alone decides; such ties are counted and must stay rare.  Weights are
compared within 1e-5 relative (float32 bulk) or 1e-4 (split-bfloat16 bulk),
log-determinants within 1e-9.
"""
import sys

import numpy as np
import pytest

from oracle import brute, sampler
from paper_2109_07358_amd import workloads

pytestmark = pytest.mark.gpu

TIE = 1e-9


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


def run(ffs, plan, seed, first, n, logdet=False):
    import torch
    x, ld = ffs.ffs_sample(plan, seed, first, n, logdet=logdet)
    torch.cuda.synchronize()
    st = ffs.ffs_check(plan)
    return x.cpu().numpy(), (ld.cpu().numpy() if ld is not None else None), st


def compare(U, X, seed, first, idx=None, n_keep=None):
    """Compare GPU rows X[idx] with the oracle; returns (n_equal, n_tie)."""
    idx = range(len(X)) if idx is None else idx
    eq = tie = 0
    for i in idx:
        r = sampler.sample_one(U, seed, first + i, n_keep)
        ref = np.array(r["x"])
        got = X[i][: len(ref)]
        if np.array_equal(got, ref):
            eq += 1
            continue
        k = int(np.argmax(got != ref))
        assert r["margin"][k] < TIE, (
            "sample %d step %d: gpu %d oracle %d, oracle margin %.3e"
            % (first + i, k, got[k], ref[k], r["margin"][k]))
        tie += 1
    return eq, tie


def check_valid(X, L):
    assert X.min() >= 0 and X.max() < L
    for row in X:
        assert len(set(row.tolist())) == len(row)


# ---------------------------------------------------------------- plain --
@pytest.mark.parametrize("bulk", ["fp64", "fp32"])
def test_plain_matches_oracle_64x16(ffs, bulk):
    say("case plain", bulk, "L=64 N=16 n=400")
    U = workloads.gaussian_qr(64, 16, 0)
    plan = ffs.ffs_plan(U, bulk=bulk, path="plain")
    X, ld, st = run(ffs, plan, 0xC1, 0, 400, logdet=True)
    check_valid(X, 64)
    eq, tie = compare(U, X, 0xC1, 0)
    say("  equal", eq, "ties", tie, "stats", st)
    assert eq + tie == 400 and tie <= 2
    for i in range(20):
        _, l = np.linalg.slogdet(U[X[i]])
        assert abs(ld[i] - 2 * l) < 1e-9 * max(1, abs(l))


def test_plain_complex_matches_oracle(ffs):
    say("case plain complex L=96 N=20")
    U = workloads.gaussian_qr(96, 20, 7, complex_=True)
    plan = ffs.ffs_plan(U, path="plain")
    X, _, st = run(ffs, plan, 3, 0, 100)
    eq, tie = compare(U, X, 3, 0)
    say("  equal", eq, "ties", tie, "stats", st)
    assert eq + tie == 100 and tie <= 1


# -------------------------------------------------------------- batched --
def test_batched_tiny_8x3(ffs):
    say("case batched L=8 N=3 n=2000")
    U = workloads.gaussian_qr(8, 3, 1)
    plan = ffs.ffs_plan(U)
    X, _, st = run(ffs, plan, 0x5EED, 0, 2000)
    check_valid(X, 8)
    eq, tie = compare(U, X, 0x5EED, 0)
    say("  equal", eq, "ties", tie, "stats", st)
    assert eq + tie == 2000 and tie <= 2


@pytest.mark.parametrize("bulk", ["fp32", "split_bf16"])
@pytest.mark.parametrize("cplx", [False, True])
def test_batched_ragged_matches_oracle(ffs, cplx, bulk):
    # L and S not multiples of the tile, N not a multiple of 16
    say("case batched ragged L=300 N=40 n=300 complex", cplx, "bulk", bulk)
    U = workloads.gaussian_qr(300, 40, 4, complex_=cplx)
    plan = ffs.ffs_plan(U, bulk=bulk)
    X, ld, st = run(ffs, plan, 77, 1000, 300, logdet=True)
    check_valid(X, 300)
    eq, tie = compare(U, X, 77, 1000)
    say("  equal", eq, "ties", tie, "stats", st)
    assert eq + tie == 300 and tie <= 2
    for i in range(10):
        _, l = np.linalg.slogdet(U[X[i]])
        assert abs(ld[i] - 2 * l) < 1e-8 * max(1, abs(l))


@pytest.mark.parametrize("cplx", [False, True])
def test_every_draw_redrawn_in_float64(ffs, cplx):
    """guard_delta = 1 flags every draw, so every site comes from the float64
    redraw: the 256-sample half-batch fills eight column tiles of the redraw
    product per step, the 14-sample one a tile whose second 16-column half is
    empty; ragged L."""
    say("case all-flagged L=1000 N=40 n=270 complex", cplx)
    U = workloads.gaussian_qr(1000, 40, 8, complex_=cplx)
    plan = ffs.ffs_plan(U, guard_delta=1.0)
    X, ld, st = run(ffs, plan, 31, 500, 270, logdet=True)
    say("  stats", st)
    check_valid(X, 1000)
    assert st["device_status"] == 0 and st["flagged"] == st["draws"] == 270 * 40
    eq, tie = compare(U, X, 31, 500, idx=range(0, 270, 3))
    say("  equal", eq, "ties", tie)
    assert eq + tie == 90 and tie <= 1
    for i in (0, 134, 135, 269):
        _, l = np.linalg.slogdet(U[X[i]])
        assert abs(ld[i] - 2 * l) < 1e-8 * max(1, abs(l))


def test_kernel_timing_hook_counts_launches(ffs):
    """ffs_set_timing / ffs_set_timing_classes: per-class launch counts of a
    two-half call (the contraction's events bound to its dispatches), times
    positive and below the call's wall time, results unchanged."""
    import time
    import torch
    say("case timing hook L=500 N=40 n=300")
    U = workloads.gaussian_qr(500, 40, 6)
    plan = ffs.ffs_plan(U, resolve="per_step")
    X0, _, _ = run(ffs, plan, 5, 0, 300)
    ffs.ffs_kernel_times(plan)  # clear
    ffs.ffs_set_timing(plan, True)
    t = time.perf_counter()
    X1, _, _ = run(ffs, plan, 5, 0, 300)
    wall_ms = (time.perf_counter() - t) * 1e3
    kt = ffs.ffs_kernel_times(plan)
    say("  times", kt)
    assert np.array_equal(X0, X1)
    n_blocks = (40 - 1) // 16  # blocks closed before the last step
    assert kt["weights"][1] == 2 * 40 and kt["draw"][1] == 2 * 40 and kt["repair"][1] == 2 * 40
    assert kt["factor"][1] + kt["factor_block"][1] == 2 * (40 + 1)
    assert kt["factor_block"][1] == 2 * n_blocks
    for c in ("weights", "draw", "repair", "factor", "factor_block"):
        assert 0.0 < kt[c][0] < wall_ms
    ffs.ffs_set_timing_classes(plan, ["weights"])
    X2, _, _ = run(ffs, plan, 5, 0, 300)
    kt = ffs.ffs_kernel_times(plan)
    assert np.array_equal(X0, X2)
    assert kt["weights"][1] == 2 * 40 and kt["weights"][0] > 0.0
    assert all(kt[c][1] == 0 for c in ("factor", "draw", "repair", "factor_block"))
    # one contraction launch in 6 bracketed (80 launches: 0, 6, ..., 78),
    # with its device span
    ffs.ffs_kernel_spans(plan)
    ffs.ffs_set_timing_stride(plan, 6)
    X3, _, _ = run(ffs, plan, 5, 0, 300)
    kt = ffs.ffs_kernel_times(plan)
    span_ms, span_n = ffs.ffs_kernel_spans(plan)
    assert np.array_equal(X0, X3)
    assert kt["weights"][1] == 14 and kt["weights"][0] > 0.0 and span_n == 14
    ffs.ffs_set_timing_stride(plan, 1)
    ffs.ffs_set_timing(plan, False)
    run(ffs, plan, 5, 0, 300)
    assert all(v[1] == 0 for v in ffs.ffs_kernel_times(plan).values())
    torch.cuda.synchronize()
    # deferred resolution: one draw + factor launch per step and half, and
    # one bracketed end-of-call check per half
    plan = ffs.ffs_plan(U, resolve="deferred")
    ffs.ffs_set_timing(plan, True)
    X4, _, _ = run(ffs, plan, 5, 0, 300)
    kt = ffs.ffs_kernel_times(plan)
    assert np.array_equal(X0, X4)
    assert kt["weights"][1] == 2 * 40 and kt["draw"][1] == 0 and kt["repair"][1] == 2
    assert kt["factor"][1] + kt["factor_block"][1] == 2 * (40 + 1)
    torch.cuda.synchronize()


def test_batched_anderson_full_size_sampled(ffs):
    """The benchmark's launch: L=4096, N=256, S=4096, sampled rows."""
    say("case batched anderson L=4096 N=256 S=4096")
    U = workloads.anderson_chain(4096, 256, 2.0, 2)
    plan = ffs.ffs_plan(U)
    X, ld, st = run(ffs, plan, 0x5EED, 0, 4096, logdet=True)
    say("  stats", st)
    check_valid(X, 4096)
    idx = [0, 1, 517, 1024, 2047, 3000, 4095]
    eq, tie = compare(U, X, 0x5EED, 0, idx)
    say("  equal", eq, "ties", tie)
    assert eq + tie == len(idx) and tie <= 1
    assert st["device_status"] == 0


@pytest.mark.parametrize("L,N,cplx", [(4096, 1024, False), (8192, 512, True)])
def test_batched_large_n_full_length(ffs, L, N, cplx):
    """Every step of N = 1024 (real) / 512 (complex) samples: log|det U[x,:]|^2
    identity on whole samples, oracle marginal on a prefix."""
    say("case full-length L=%d N=%d complex %s S=130" % (L, N, cplx))
    U = workloads.gaussian_qr(L, N, 12, complex_=cplx)
    plan = ffs.ffs_plan(U)
    X, ld, st = run(ffs, plan, 21, 0, 130, logdet=True)
    say("  stats", st)
    assert st["device_status"] == 0
    check_valid(X, L)
    for i in (0, 64, 129):
        _, l = np.linalg.slogdet(U[X[i]])
        assert abs(ld[i] - 2 * l) < 1e-7 * max(1.0, abs(l)), (i, ld[i], 2 * l)
    eq, tie = compare(U, X, 21, 0, [0, 129], n_keep=48)
    assert eq + tie == 2 and tie <= 1


def test_split_bf16_anderson_full_size_sampled(ffs):
    """Split-bfloat16 contraction at L=4096, N=256, S=4096, sampled rows."""
    say("case split-bf16 anderson L=4096 N=256 S=4096")
    U = workloads.anderson_chain(4096, 256, 2.0, 2)
    plan = ffs.ffs_plan(U, bulk="split_bf16")
    X, _, st = run(ffs, plan, 0x5EED, 0, 4096)
    say("  stats", st)
    check_valid(X, 4096)
    idx = [0, 1, 517, 2047, 4095]
    eq, tie = compare(U, X, 0x5EED, 0, idx)
    say("  equal", eq, "ties", tie)
    assert eq + tie == len(idx) and tie <= 1
    assert st["device_status"] == 0 and st["flagged"] > 0


# --------------------------------------------------- invariances, hooks --
def test_marginal_is_prefix_and_split_invariant(ffs):
    import torch
    say("case marginal/split L=200 N=24")
    U = workloads.gaussian_qr(200, 24, 5)
    plan = ffs.ffs_plan(U)
    small = ffs.ffs_plan(U, max_batch=128)
    X, _, _ = run(ffs, plan, 9, 0, 300)
    parts = [run(ffs, plan, 9, a, 100)[0] for a in (0, 100, 200)]
    assert np.array_equal(X, np.concatenate(parts))
    Y, _, _ = run(ffs, small, 9, 0, 300)
    assert np.array_equal(X, Y)
    one = ffs.ffs_plan(U, overlap=False)  # one stream, no half-batch split
    Z, _, _ = run(ffs, one, 9, 0, 300)
    assert np.array_equal(X, Z)
    M = ffs.ffs_marginal(plan, 7, 9, 0, 300)
    torch.cuda.synchronize()
    assert np.array_equal(M.cpu().numpy(), X[:, :7])
    pl = ffs.ffs_plan(U, path="plain")
    Mp = ffs.ffs_marginal(pl, 7, 9, 0, 50)
    torch.cuda.synchronize()
    assert np.array_equal(Mp.cpu().numpy(), X[:50, :7])


@pytest.mark.parametrize("cplx", [False, True])
def test_tile_variants_are_bit_identical(ffs, cplx):
    """Every contraction tile gives the same draws and log-determinants, and
    the autotuner's choice is one of them."""
    say("case tile variants complex", cplx)
    U = workloads.gaussian_qr(1000, 96, 13, complex_=cplx)
    plan = ffs.ffs_plan(U)
    n = 300
    shapes = [(128, 128), (64, 128)] + ([] if cplx else [(128, 64), (64, 64)])
    tiles = [(tm, tn, kc) for kc in (32, 16) for tm, tn in shapes]
    ref = None
    for tm, tn, kc in tiles:
        ffs.ffs_set_tile(plan, n, tm, tn, kc)
        X, ld, _ = run(ffs, plan, 8, 0, n, logdet=True)
        if ref is None:
            ref = (X, ld)
        assert np.array_equal(X, ref[0]) and np.array_equal(ld, ref[1]), (tm, tn, kc)
    for pipeline in (False, True):
        choice = ffs.ffs_autotune(plan, n, pipeline=pipeline)
        say("  autotune choice", choice, "pipeline", pipeline)
        assert ffs.parse_tile(choice) in tiles
    X, ld, _ = run(ffs, plan, 8, 0, n, logdet=True)
    assert np.array_equal(X, ref[0])


# float32 bulk: 1e-5 relative; split-bfloat16 bulk: its stated 1e-4 (three
# bfloat16 products carry about 2^-16 relative each; measured <= 2.5e-5)
WEIGHT_TOL = {"fp32": 1e-5, "split_bf16": 1e-4}


@pytest.mark.parametrize("bulk", ["fp32", "split_bf16"])
@pytest.mark.parametrize("cplx", [False, True])
def test_conditional_weights_within_tolerance(ffs, cplx, bulk):
    say("case teacher-forced weights complex", cplx, "bulk", bulk)
    L, N = 300, 40
    U = workloads.gaussian_qr(L, N, 6, complex_=cplx)
    plan = ffs.ffs_plan(U, bulk=bulk)
    ref_x = sampler.sample_one(U, 5, 2)["x"]
    for k in (1, 2, 9, 25, 40):
        w = ffs.ffs_conditional(plan, 5, 2, ref_x[: k - 1])
        ref = sampler.teacher_forced_weights(U, 5, 2, ref_x[: k - 1])
        floor = 1.0 / (L - k + 1)
        err = np.max(np.abs(w - ref) / np.maximum(ref, floor))
        say("  k", k, "max rel err", err)
        assert err < WEIGHT_TOL[bulk]
        assert np.all(w[ref_x[: k - 1]] == 0.0)


@pytest.mark.parametrize("bulk", ["fp32", "split_bf16"])
def test_global_phase_leaves_draws_unchanged(ffs, bulk):
    """|det((e^{i theta} Q)[x, :])|^2 = |det Q[x, :]|^2 (Eq. (1)): the complex
    path on U = e^{i theta} Q, Q real, must draw what the oracle draws for Q
    itself (same Philox stream, so the same column orders), with the same
    log-determinants and weights.  The phases make U real (Ui = 0), purely
    imaginary (Ur = 0), nearly cancelling in Ur + Ui (the third product of
    the complex contraction's three then carries almost nothing), and
    generic."""
    L, N, n, seed = 700, 72, 64, 21
    Q = workloads.gaussian_qr(L, N, 17)
    refs = [sampler.sample_one(Q, seed, i) for i in range(n)]
    for theta in (0.0, np.pi / 2, 3 * np.pi / 4 + 0.01, 2.0):
        say("case global phase", theta, "bulk", bulk)
        plan = ffs.ffs_plan(np.exp(1j * theta) * Q, bulk=bulk)
        X, LD, st = run(ffs, plan, seed, 0, n, logdet=True)
        check_valid(X, L)
        ties = 0
        for i, r in enumerate(refs):
            ref = np.array(r["x"])
            if np.array_equal(X[i], ref):
                assert abs(LD[i] - r["logdet"]) < 1e-9 * max(1.0, abs(r["logdet"])), i
                continue
            k = int(np.argmax(X[i] != ref))
            assert r["margin"][k] < TIE, (
                "theta %g sample %d step %d: gpu %d oracle %d, oracle margin %.3e"
                % (theta, i, k, X[i][k], ref[k], r["margin"][k]))
            ties += 1
        assert ties <= 1 and st["device_status"] == 0
        pre = refs[3]["x"]
        for k in (1, 30, N):
            w = ffs.ffs_conditional(plan, seed, 3, pre[: k - 1])
            ref = sampler.teacher_forced_weights(Q, seed, 3, pre[: k - 1])
            err = np.max(np.abs(w - ref) / np.maximum(ref, 1.0 / (L - k + 1)))
            say("  k", k, "max rel err", err)
            assert err < WEIGHT_TOL[bulk]
        ffs.ffs_destroy(plan)


def test_density(ffs):
    U = workloads.gaussian_qr(500, 50, 8, complex_=True)
    plan = ffs.ffs_plan(U)
    rho = ffs.ffs_density(plan)
    ref = sampler.density(U)
    assert np.max(np.abs(rho - ref)) < 1e-6
    assert abs(rho.sum() - 50) < 1e-4


def test_gpu_samples_follow_eq1_law(ffs):
    from scipy import stats
    say("case chi-square L=8 N=3 n=200000")
    U = workloads.gaussian_qr(8, 3, 1)
    law = brute.set_law(brute.det_law(U))
    keys = sorted(law)
    plan = ffs.ffs_plan(U)
    X, _, _ = run(ffs, plan, 123, 0, 200000)
    code = {k: i for i, k in enumerate(keys)}
    S = np.sort(X, axis=1)
    obs = np.zeros(len(keys))
    for row in map(tuple, S):
        obs[code[row]] += 1
    exp = np.array([law[k] for k in keys]) * len(X)
    p = stats.chisquare(obs, exp).pvalue
    say("  p-value", p)
    assert p > 1e-4


def test_gpu_site_marginals_match_density(ffs):
    say("case site marginals L=4096 N=256 anderson n=4096")
    U = workloads.anderson_chain(4096, 256, 2.0, 2)
    plan = ffs.ffs_plan(U)
    X, _, _ = run(ffs, plan, 4, 0, 4096)
    rho = sampler.density(U)
    freq = np.bincount(X.ravel(), minlength=4096) / len(X)
    sd = np.sqrt(np.maximum(rho * (1 - rho), 1e-12) / len(X))
    z = (freq - rho) / sd
    ok = rho > 1e-3
    say("  max |z|", np.max(np.abs(z[ok])))
    assert np.max(np.abs(z[ok])) < 6.0
    assert abs(freq.sum() - 256) < 1e-9


@pytest.mark.parametrize("cplx", [False, True])
def test_gpu_pair_function_matches_kernel(ffs, cplx):
    """Two-point function of the determinantal law: P(i and j occupied) =
    rho_i rho_j - |K_ij|^2 with K = U U^dagger (z-scores over all pairs)."""
    say("case pair function L=24 N=6 complex=%s n=200000" % cplx)
    U = workloads.gaussian_qr(24, 6, 21, complex_=cplx)
    plan = ffs.ffs_plan(U)
    X, _, _ = run(ffs, plan, 321, 0, 200000)
    n = len(X)
    occ = np.zeros((n, 24), dtype=np.float64)
    occ[np.arange(n)[:, None], X] = 1.0
    pair = occ.T @ occ / n
    K = U @ U.conj().T
    rho = np.real(np.diag(K))
    want = np.outer(rho, rho) - np.abs(K) ** 2
    iu = np.triu_indices(24, 1)
    p, q = want[iu], pair[iu]
    ok = p > 1e-3
    z = (q[ok] - p[ok]) / np.sqrt(p[ok] * (1 - p[ok]) / n)
    say("  pairs", int(ok.sum()), "max |z|", float(np.abs(z).max()))
    assert np.abs(z).max() < 6.0
    assert np.allclose(np.diag(pair), rho, atol=6 * np.sqrt(0.25 / n))


def test_complex_c3_launch_shape_sampled(ffs):
    """Complex L=16384, N=512, S=8192 (the contraction target shape): first
    12 steps of every sample; sampled rows against the oracle's marginal."""
    import torch
    say("case complex L=16384 N=512 S=8192 marginal 12")
    U = workloads.gaussian_qr(16384, 512, 3, complex_=True)
    plan = ffs.ffs_plan(U)
    M = ffs.ffs_marginal(plan, 12, 11, 0, 8192)
    torch.cuda.synchronize()
    st = ffs.ffs_check(plan)
    X = M.cpu().numpy()
    check_valid(X, 16384)
    idx = [0, 63, 64, 4000, 8191]
    eq, tie = compare(U, X, 11, 0, idx, n_keep=12)
    say("  equal", eq, "ties", tie, "stats", st)
    assert eq + tie == len(idx) and tie <= 1
