"""GPU tests of the request server: every result of a mixed, concurrently
running set of requests equals the same call made alone (bit-exact), and
sampled requests equal the oracle."""
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


@pytest.mark.parametrize("mode", ["grouped", "streams"])
def test_server_mix_equals_alone(ffs, mode):
    import torch
    say("case server mix: 4 plans (one split-bf16), 24 requests, tight budget, mode", mode)
    Us = [workloads.gaussian_qr(300, 40, 4),
          workloads.gaussian_qr(500, 24, 8, complex_=True),
          workloads.anderson_chain(1024, 64, 2.0, 2),
          workloads.gaussian_qr(600, 32, 18)]
    plans = [ffs.ffs_plan(U, bulk="split_bf16" if j == 3 else "fp32") for j, U in enumerate(Us)]
    rng = np.random.default_rng(11)
    reqs = []
    for i in range(24):
        j = int(rng.integers(0, 4))
        N = Us[j].shape[1]
        n = int(rng.integers(1, 260))
        n_keep = N if i % 3 else int(rng.integers(1, N + 1))
        reqs.append((j, n_keep, int(rng.integers(0, 2 ** 40)), int(rng.integers(0, 2 ** 30)), n))
    # budget: room for about two of the largest requests at once
    srv = ffs.Server(mode=mode, slots=4, capacity=6, ticks=8, hbm_budget=200 << 20)
    outs = [torch.full((n, n_keep), -1, dtype=torch.int32, device="cuda")
            for (j, n_keep, seed, first, n) in reqs]
    torch.cuda.synchronize()  # the server's streams do not wait for torch's
    tickets = [srv.submit(plans[j], n_keep, seed, first, n, x)
               for (j, n_keep, seed, first, n), x in zip(reqs, outs)]
    infos = [srv.poll(t, timeout_ms=-1) for t in tickets]
    srv.close()
    for inf in infos:
        assert inf["state"] == "done" and inf["status"] == 0, inf
        assert inf["t_submit"] <= inf["t_admit"] <= inf["t_done"]
    # requests overlapped on the device
    spans = sorted((inf["t_admit"], inf["t_done"]) for inf in infos)
    overlap = any(spans[k + 1][0] < spans[k][1] for k in range(len(spans) - 1))
    assert overlap
    torch.cuda.synchronize()
    for (j, n_keep, seed, first, n), x, inf in zip(reqs, outs, infos):
        alone = ffs.ffs_marginal(plans[j], n_keep, seed, first, n)
        torch.cuda.synchronize()
        assert np.array_equal(x.cpu().numpy(), alone.cpu().numpy()), (j, n_keep, n)
        assert inf["draws"] == n * n_keep
    # two requests against the oracle
    for (j, n_keep, seed, first, n), x in list(zip(reqs, outs))[:2]:
        X = x.cpu().numpy()
        for i in (0, n - 1):
            ref = sampler.sample_one(Us[j], seed, first + i, n_keep)
            if not np.array_equal(X[i], ref["x"]):
                k = int(np.argmax(X[i] != np.array(ref["x"])))
                assert ref["margin"][k] < 1e-9
    say("  ok; spans", len(spans))


def test_server_grouped_admits_while_running(ffs):
    """A request submitted while a long one runs finishes before it."""
    import torch
    say("case grouped admission mid-run")
    long_U = workloads.gaussian_qr(4096, 256, 9)
    short_U = workloads.gaussian_qr(300, 40, 4)
    pl, ps = ffs.ffs_plan(long_U), ffs.ffs_plan(short_U)
    xl = torch.empty((512, 256), dtype=torch.int32, device="cuda")
    xs = torch.empty((8, 40), dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    srv = ffs.Server(mode="grouped", capacity=4, ticks=4)
    tl = srv.submit(pl, 256, 3, 0, 512, xl)
    import time
    time.sleep(0.01)
    ts = srv.submit(ps, 40, 4, 0, 8, xs)
    i_s = srv.poll(ts, -1)
    i_l = srv.poll(tl, -1)
    srv.close()
    assert i_s["t_admit"] < i_l["t_done"] and i_s["t_done"] < i_l["t_done"]
    torch.cuda.synchronize()
    a = ffs.ffs_sample(pl, 3, 0, 512)[0]
    b = ffs.ffs_sample(ps, 4, 0, 8)[0]
    torch.cuda.synchronize()
    assert np.array_equal(xl.cpu().numpy(), a.cpu().numpy())
    assert np.array_equal(xs.cpu().numpy(), b.cpu().numpy())


def test_server_rejects_request_over_budget(ffs):
    import torch
    from paper_2109_07358_amd.ffs import FFSError
    U = workloads.gaussian_qr(300, 40, 4)
    plan = ffs.ffs_plan(U)
    srv = ffs.Server(slots=1, hbm_budget=1 << 20)
    x = torch.empty((100, 40), dtype=torch.int32, device="cuda")
    with pytest.raises(FFSError):
        srv.submit(plan, 40, 1, 0, 100, x)
    srv.close()
