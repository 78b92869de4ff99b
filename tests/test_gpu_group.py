"""GPU tests of grouped runs: instances of uneven L, N, sample counts and
n_keep advanced in lockstep (direct launches and replayed hipGraphs) give
exactly the results of the separate calls."""
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


@pytest.fixture(scope="module")
def plans(ffs):
    Us = [workloads.gaussian_qr(300, 40, 4),
          workloads.gaussian_qr(500, 24, 8, complex_=True),
          workloads.anderson_chain(1024, 64, 2.0, 2),
          workloads.gaussian_qr(4096, 256, 9)]
    return Us, [ffs.ffs_plan(U) for U in Us]


def _items(ffs, plans, spec):
    import torch
    Us, ps = plans
    items = []
    for j, n, n_keep, seed, first, with_ld in spec:
        it = {"plan": ps[j], "n_keep": n_keep, "seed": seed, "first_sample": first,
              "n_samples": n,
              "x_out": torch.full((n, n_keep), -1, dtype=torch.int32, device="cuda")}
        if with_ld:
            it["logdet_out"] = torch.zeros(n, dtype=torch.float64, device="cuda")
        items.append(it)
    return items


def _check_alone(ffs, items):
    import torch
    torch.cuda.synchronize()
    for it in items:
        if "logdet_out" in it:
            x, ld = ffs.ffs_sample(it["plan"], it["seed"], it["first_sample"],
                                   it["n_samples"], logdet=True)
            torch.cuda.synchronize()
            assert np.array_equal(it["logdet_out"].cpu().numpy(), ld.cpu().numpy())
        else:
            x = ffs.ffs_marginal(it["plan"], it["n_keep"], it["seed"],
                                 it["first_sample"], it["n_samples"])
            torch.cuda.synchronize()
        assert np.array_equal(it["x_out"].cpu().numpy(), x.cpu().numpy())


SPEC = [(0, 100, 40, 5, 0, True), (1, 37, 10, 6, 100, False),
        (2, 200, 64, 7, 0, False), (3, 130, 20, 8, 9, False),
        (0, 1, 3, 9, 77, False), (1, 129, 24, 10, 0, True)]


@pytest.mark.parametrize("graph", [False, True])
def test_group_equals_separate_calls(ffs, plans, graph):
    import torch
    say("case group of 6 instances, graph", graph)
    items = _items(ffs, plans, SPEC)
    torch.cuda.synchronize()
    st = ffs.ffs_sample_group(items, graph=graph, stats=True)
    for it, s in zip(items, st):
        assert s["device_status"] == 0
        assert s["draws"] == it["n_samples"] * it["n_keep"]
    _check_alone(ffs, items)
    # two sampled rows against the oracle
    Us = plans[0]
    X = items[2]["x_out"].cpu().numpy()
    for i in (0, 199):
        ref = sampler.sample_one(Us[2], 7, i, 64)
        if not np.array_equal(X[i], ref["x"]):
            k = int(np.argmax(X[i] != np.array(ref["x"])))
            assert ref["margin"][k] < 1e-9


def test_group_graph_replays_across_calls(ffs, plans):
    """Graph mode twice in a row with eager work between the calls; every
    replay (several per call) is checked against the separate calls."""
    import torch
    say("case group graph twice")
    a = _items(ffs, plans, SPEC)
    torch.cuda.synchronize()
    ffs.ffs_sample_group(a, graph=True)
    _check_alone(ffs, a)
    b = _items(ffs, plans, [(3, 64, 40, 21, 5, False), (2, 33, 17, 22, 0, False),
                            (0, 260, 40, 23, 1, True)])
    torch.cuda.synchronize()
    ffs.ffs_sample_group(b, graph=True)
    _check_alone(ffs, b)


def test_group_with_split_bf16_plans(ffs, plans):
    """Split-BF16 plans (real and complex) in a group with an FP32 plan, direct
    and as a replayed graph: each instance equals its separate call."""
    import torch
    say("case group with split-bf16 plans")
    Us = [workloads.gaussian_qr(700, 48, 16), workloads.gaussian_qr(400, 20, 17, complex_=True)]
    bp = [ffs.ffs_plan(U, bulk="split_bf16") for U in Us]
    mixed = (Us + plans[0][:1], bp + plans[1][:1])
    for graph in (False, True):
        items = _items(ffs, mixed, [(0, 150, 48, 31, 0, True), (1, 60, 20, 32, 5, False),
                                    (2, 90, 40, 33, 1, False), (1, 129, 20, 34, 7, True)])
        torch.cuda.synchronize()
        st = ffs.ffs_sample_group(items, graph=graph, stats=True)
        say("  graph", graph, "stats", st)
        for it, s in zip(items, st):
            assert s["device_status"] == 0 and s["draws"] == it["n_samples"] * it["n_keep"]
        _check_alone(ffs, items)
