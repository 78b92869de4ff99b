"""bench.py's host-side contract: one GPU only, traffic figures tied to the
kernel sources they were measured on, and the factor byte model."""
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_only_for_the_measured_sources():
    b = _bench()
    for tile in b.MEASURED_TRAFFIC["weights"]["tiles"]:
        assert b.measured_traffic("weights", tile) == b.MEASURED_TRAFFIC["weights"]["tiles"][tile]
    assert b.measured_traffic("weights", "32x32") is None
    b.MEASURED_TRAFFIC["weights"]["sources"] = {"k_weights.hip": "0000000000000000"}
    assert b.measured_traffic("weights", "64x64") is None


def test_factor_byte_model():
    b = _bench()
    one = b.factor_bytes(4096, 256, 1, 8, 256)
    assert one > 0
    # linear in the samples, growing faster than linearly in N
    assert b.factor_bytes(4096, 256, 4096, 8, 256) == 4096 * one
    assert b.factor_bytes(4096, 512, 1, 8, 512) > 4 * one
    # complex entries double the bytes of the entry-sized terms
    assert b.factor_bytes(4096, 256, 1, 16, 256) > one
