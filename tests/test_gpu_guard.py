"""Soundness of the near-tie guard where it runs (Eq. (2)'s inverse-CDF draw).

The guard redraws in float64 every draw whose reduced-precision CDF puts u*T
within its threshold of a site boundary; a draw it leaves alone is kept
from the float32 (or split-bfloat16) weights.  guard_delta = 1 flags every
draw, so that run's sites all come from float64 weights.  With the default
(adaptive) threshold the two runs must agree draw for draw -- any difference
would be an unflagged draw that float64 places elsewhere -- on the
benchmark's chain launch (1,048,576 draws) and on the complex L=16384 N=512
launch shape (1,024 complete samples, 524,288 draws), float32 and
split-bfloat16.  The default float32 flag rate at that complex shape stays
below 1%."""
import sys

import numpy as np
import pytest

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


def _default_vs_float64(ffs, U, bulk, seed, S):
    import torch
    ref = ffs.ffs_plan(U, bulk=bulk, guard_delta=1.0)
    R = ffs.ffs_sample(ref, seed, 0, S)[0]
    torch.cuda.synchronize()
    sr = ffs.ffs_check(ref)
    assert sr["flagged"] == sr["draws"]
    R = R.cpu().numpy()
    del ref
    torch.cuda.empty_cache()
    plan = ffs.ffs_plan(U, bulk=bulk)
    X = ffs.ffs_sample(plan, seed, 0, S)[0]
    torch.cuda.synchronize()
    st = ffs.ffs_check(plan)
    X = X.cpu().numpy()
    bad = np.nonzero((X != R).any(axis=1))[0]
    say("  default guard: %d of %d draws flagged (%.3f%%), %d samples differ from the "
        "all-float64 run" % (st["flagged"], st["draws"], 100.0 * st["flagged"] / st["draws"],
                             len(bad)))
    assert st["device_status"] == 0 and len(bad) == 0, [
        (int(i), int(np.argmax(X[i] != R[i]))) for i in bad[:5]]
    return st


@pytest.mark.parametrize("bulk", ["fp32", "split_bf16"])
def test_guard_chain_benchmark_launch(ffs, bulk):
    say("case guard chain L=4096 N=256 S=4096", bulk)
    U = workloads.anderson_chain(4096, 256, 2.0, 2)
    _default_vs_float64(ffs, U, bulk, 0x5EED, 4096)


@pytest.mark.parametrize("bulk", ["fp32", "split_bf16"])
def test_guard_complex_launch_shape(ffs, bulk):
    say("case guard complex L=16384 N=512 S=1024", bulk)
    U = workloads.gaussian_qr(16384, 512, 3, complex_=True)
    st = _default_vs_float64(ffs, U, bulk, 21, 1024)
    if bulk == "fp32":
        assert st["flagged"] < 0.01 * st["draws"]
