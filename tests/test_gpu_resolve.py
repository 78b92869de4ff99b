"""Deferred resolution of flagged draws against per-step resolution.

Both modes give every flagged draw the site of its float64 weights with the
draw's own uniform; deferred resolution only moves that work to the end of
the call (one float64 check per recorded draw) and replays, per step, the
samples whose recorded site moved or whose record found no slot.  So the
two modes must give identical configurations and log-determinants, element
by element.  The cases cover: no replay (the usual case), every sample
replayed because the record pool overflows, and replays caused by moved
sites (split-bfloat16 weights with every draw flagged and the pool large
enough to hold every record), plus marginals, ragged batches and a
comparison of the replayed samples with the oracle.
"""
import sys

import numpy as np
import pytest

from oracle import sampler
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


def run(ffs, plan, seed, first, n, n_keep=None):
    import torch
    if n_keep is None:
        x, ld = ffs.ffs_sample(plan, seed, first, n, logdet=True)
    else:
        x = ffs.ffs_marginal(plan, n_keep, seed, first, n)
        ld = None
    torch.cuda.synchronize()
    st = ffs.ffs_check(plan)
    return x.cpu().numpy(), (ld.cpu().numpy() if ld is not None else None), st


def both(ffs, U, seed, first, n, n_keep=None, **kw):
    p1 = ffs.ffs_plan(U, resolve="per_step", **kw)
    X1, L1, s1 = run(ffs, p1, seed, first, n, n_keep)
    del p1
    p2 = ffs.ffs_plan(U, resolve="deferred", **kw)
    X2, L2, s2 = run(ffs, p2, seed, first, n, n_keep)
    say("  per-step", s1, "deferred", s2)
    assert s1["device_status"] == 0 and s2["device_status"] == 0
    assert np.array_equal(X1, X2), np.argwhere((X1 != X2).any(axis=1))[:5].ravel()
    if L1 is not None:
        assert np.array_equal(L1, L2)
    return X1, s1, s2


def test_auto_mode_is_deferred_for_fp32_default_guard(ffs):
    # (no call here needs a replay, which would turn a plan per step)
    say("case auto resolution L=700 N=40 n=300")
    U = workloads.gaussian_qr(700, 40, 4)
    for kw, want in (({}, 2), ({"guard_delta": 1e-3}, 1), ({"bulk": "split_bf16"}, 1),
                     ({"guard_scale": 16.0}, 1), ({"guard_scale": 4.0}, 2)):
        plan = ffs.ffs_plan(U, **kw)
        assert plan.options.resolve == 0
        # the mode actually taken shows in the launch counts of a timed call
        ffs.ffs_set_timing(plan, True)
        run(ffs, plan, 3, 0, 300)
        kt = ffs.ffs_kernel_times(plan)
        got = 2 if kt["draw"][1] == 0 else 1
        say("  options", kw, "mode", got)
        assert got == want


def test_deferred_equals_per_step_without_replays(ffs):
    # ragged L and batch, two half-batches; the default guard flags a few
    # draws, none moves
    say("case deferred L=2000 N=96 n=700")
    U = workloads.gaussian_qr(2000, 96, 11)
    X, s1, s2 = both(ffs, U, 0xD1, 33, 700)
    assert s1["changed"] == 0 and s2["changed"] == 0
    assert s2["flagged"] == s1["flagged"]


def test_deferred_marginal_and_complex(ffs):
    say("case deferred marginal L=900 N=50 n_keep=37 n=260 complex")
    U = workloads.gaussian_qr(900, 50, 12, complex_=True)
    both(ffs, U, 0xD2, 0, 260, n_keep=37)
    X, _, _ = both(ffs, U, 0xD2, 0, 260)


def test_record_overflow_replays_every_sample(ffs):
    # a fixed margin of 1 flags every draw: the pool (two records per
    # sample at N = 40) fills in the first steps and every sample is then
    # listed and replayed per step; the result is the all-float64 run
    say("case deferred overflow L=1000 N=40 n=270")
    U = workloads.gaussian_qr(1000, 40, 8)
    X, s1, s2 = both(ffs, U, 31, 500, 270, guard_delta=1.0)
    assert s1["flagged"] == s1["draws"] == 270 * 40
    # main pass flags every draw, and every sample's replay flags its draws again
    assert s2["flagged"] == 2 * 270 * 40


def test_moved_sites_are_replayed(ffs):
    # N = 2 keeps every record in the pool (two per sample) with every draw
    # flagged; with split-bfloat16 weights at L = 65536 about one draw in
    # 800 gets another site from the bulk weights than from float64 (about
    # 20 expected here), so the end-of-call check lists those samples and
    # their replays restore the float64 sites
    say("case deferred moved sites L=65536 N=2 n=8192 split-bf16")
    U = workloads.gaussian_qr(65536, 2, 13)
    X, s1, s2 = both(ffs, U, 0xD3, 0, 8192, bulk="split_bf16", guard_delta=1.0)
    say("  changed per-step", s1["changed"], "deferred", s2["changed"])
    assert s1["changed"] > 0 and s2["changed"] >= s1["changed"]
    # the rows whose sites float64 moved are those where a run with the
    # guard off (bulk weights only) differs; each of them, and a sample of
    # the others, against the oracle
    p0 = ffs.ffs_plan(U, bulk="split_bf16", guard_scale=0.0)
    X0, _, s0 = run(ffs, p0, 0xD3, 0, 8192)
    assert s0["flagged"] == 0
    moved = np.nonzero((X0 != X).any(axis=1))[0]
    say("  rows moved by float64", len(moved))
    assert len(moved) > 0
    for i in sorted(set(moved.tolist()) | set(range(0, 8192, 512))):
        r = sampler.sample_one(U, 0xD3, i)
        ref = np.array(r["x"])
        if not np.array_equal(X[i], ref):
            k = int(np.argmax(X[i] != ref))
            assert r["margin"][k] < TIE


def test_benchmark_launch_deferred_equals_per_step(ffs):
    # the benchmark's shape, a quarter of its batch
    say("case deferred chain L=4096 N=256 n=1024")
    U = workloads.anderson_chain(4096, 256, 2.0, 2)
    both(ffs, U, 0x5EED, 2048, 1024)


def test_auto_resolution_turns_per_step_after_a_replay(ffs):
    # AUTO takes deferred resolution (float32, adaptive guard of 8 units);
    # at L = 65536, N = 256 about 2% of draws are flagged, more than the
    # pool of four records per sample holds, so the first call replays
    # samples -- and the plan resolves per step from its next call on.
    # Every call equals a per-step plan's.
    import torch
    say("case auto switch L=65536 N=256 n=256")
    U = workloads.gaussian_qr(65536, 256, 14)
    ref = ffs.ffs_plan(U, resolve="per_step", guard_scale=8.0)
    R1, _, r1 = run(ffs, ref, 0xD4, 0, 256)
    R2, _, r2 = run(ffs, ref, 0xD4, 256, 256)
    del ref
    plan = ffs.ffs_plan(U, guard_scale=8.0)
    ffs.ffs_set_timing(plan, True)
    X1, _, s1 = run(ffs, plan, 0xD4, 0, 256)
    k1 = ffs.ffs_kernel_times(plan)
    X2, _, s2 = run(ffs, plan, 0xD4, 256, 256)
    k2 = ffs.ffs_kernel_times(plan)
    say("  first call", s1, "draw launches", k1["draw"][1], "second", s2, k2["draw"][1])
    assert np.array_equal(X1, R1) and np.array_equal(X2, R2)
    assert k1["draw"][1] == 0 and s1["flagged"] > r1["flagged"]  # deferred, with replays
    assert k2["draw"][1] > 0 and s2["flagged"] == r2["flagged"]  # per step
    torch.cuda.synchronize()


def test_deferred_chunked_calls_replay_per_chunk(ffs):
    # max_batch 256: 700 samples run as chunks of 256, 256, 188, each as two
    # half-batches; every draw flagged overflows each chunk's pool, so every
    # chunk replays its samples into its own rows of the output
    say("case deferred chunked L=600 N=24 n=700 max_batch=256")
    U = workloads.gaussian_qr(600, 24, 15)
    X, s1, s2 = both(ffs, U, 0xD5, 9, 700, guard_delta=1.0, max_batch=256)
    assert s1["flagged"] == 700 * 24 and s2["flagged"] > s1["flagged"]
    # and the marginal of the same call
    both(ffs, U, 0xD5, 9, 700, n_keep=11, guard_delta=1.0, max_batch=256)


def test_deferred_calls_on_two_streams_from_two_threads(ffs):
    # a plan's calls on different streams may run concurrently: each stream
    # has its own working memory, record pool, replay batch and listed
    # counts.  Both calls here replay every sample (pool overflow).
    import threading
    import torch
    say("case deferred, two threads on two streams L=800 N=30 n=300")
    U = workloads.gaussian_qr(800, 30, 19)
    ref = ffs.ffs_plan(U, resolve="per_step", guard_delta=1.0)
    R = [run(ffs, ref, 0xD6 + k, 0, 300)[0] for k in range(2)]
    del ref
    plan = ffs.ffs_plan(U, resolve="deferred", guard_delta=1.0)
    streams = [torch.cuda.Stream() for _ in range(2)]
    outs = [torch.full((300, 30), -1, dtype=torch.int32, device="cuda") for _ in range(2)]
    torch.cuda.synchronize()
    errs = []

    def work(k):
        try:
            for _ in range(3):
                ffs.ffs_sample(plan, 0xD6 + k, 0, 300, x_out=outs[k], stream=streams[k])
            streams[k].synchronize()
        except Exception as e:  # reported below
            errs.append(e)

    th = [threading.Thread(target=work, args=(k,)) for k in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    torch.cuda.synchronize()
    assert not errs, errs
    for k in range(2):
        assert np.array_equal(outs[k].cpu().numpy(), R[k])
