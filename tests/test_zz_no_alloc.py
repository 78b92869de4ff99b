"""The allocation-free entry point (ffs_sample_noalloc) through the C ABI:
bit-identical to ffs_sample on the same plan and arguments, on consecutive
calls that reuse the library's scratch array (the second smaller than the
first, on another plan), with batches chunked to fit the array, and refused
with a clear error when one batch cannot fit."""
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


def _both(ffs, plan, seed, first, n):
    import torch
    x_ref, ld_ref = ffs.ffs_sample(plan, seed, first, n, logdet=True)
    torch.cuda.synchronize()
    st_ref = ffs.ffs_check(plan)
    x = torch.full((n, plan.N), -7, dtype=torch.int32, device="cuda")
    ld = torch.full((n,), -7.0, dtype=torch.float64, device="cuda")
    ffs.ffs_sample_noalloc(plan, seed, first, n, x, ld)
    torch.cuda.synchronize()
    st = ffs.ffs_check(plan)
    return (x_ref.cpu().numpy(), ld_ref.cpu().numpy(), st_ref,
            x.cpu().numpy(), ld.cpu().numpy(), st)


def test_noalloc_equals_sample_on_consecutive_calls(ffs):
    # first call: L=4096 N=256 -- one 128-sample batch fills about 143 MB of
    # the 256 MiB array, so 300 samples run as chunks of 128, 128, 44
    say("case noalloc chain L=4096 N=256 n=300")
    U = workloads.anderson_chain(4096, 256, 2.0, 2)
    # the allocation-free call resolves flagged draws per step (it never
    # waits for the device); with the plan in that mode the guard counters
    # match too
    plan = ffs.ffs_plan(U, resolve="per_step")
    xr, lr, sr, x, ld, st = _both(ffs, plan, 0x5EED, 17, 300)
    say("  stats", sr, st)
    assert np.array_equal(x, xr) and np.array_equal(ld, lr)
    assert st["device_status"] == 0 and st["draws"] == 300 * 256
    assert st["flagged"] == sr["flagged"] and st["changed"] == sr["changed"]
    # a default plan (deferred resolution for ffs_sample): the same sites
    plan_d = ffs.ffs_plan(U)
    xr, lr, _, x, ld, _ = _both(ffs, plan_d, 0x5EED, 17, 300)
    assert np.array_equal(x, xr) and np.array_equal(ld, lr)
    del plan_d
    # second call, smaller, another plan (complex, ragged L and N): the array
    # still holds the first call's state
    say("case noalloc complex L=500 N=40 n=70")
    U2 = workloads.gaussian_qr(500, 40, 8, complex_=True)
    plan2 = ffs.ffs_plan(U2)
    xr, lr, sr, x, ld, st = _both(ffs, plan2, 3, 0, 70)
    say("  stats", sr, st)
    assert np.array_equal(x, xr) and np.array_equal(ld, lr)
    assert st["device_status"] == 0 and st["draws"] == 70 * 40


def test_noalloc_refuses_batches_beyond_the_array(ffs):
    import torch
    say("case noalloc refusal L=2048 N=1024")
    U = workloads.gaussian_qr(2048, 1024, 2)
    plan = ffs.ffs_plan(U)
    x = torch.empty((4, 1024), dtype=torch.int32, device="cuda")
    with pytest.raises(ffs.FFSError) as e:
        ffs.ffs_sample_noalloc(plan, 1, 0, 4, x)
    assert "exceeds" in str(e.value) and e.value.status == -6
    plain = ffs.ffs_plan(workloads.gaussian_qr(64, 16, 0), path="plain")
    y = torch.empty((4, 16), dtype=torch.int32, device="cuda")
    with pytest.raises(ffs.FFSError):
        ffs.ffs_sample_noalloc(plain, 1, 0, 4, y)
    with pytest.raises(ValueError):
        ffs.ffs_sample_noalloc(plain, 1, 0, 8, y)  # output too small
