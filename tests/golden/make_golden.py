#!/usr/bin/env python3
"""Writes the stored oracle results that the full-size GPU parity tests use.

TEST INFRASTRUCTURE.  This script calls only the CPU oracle (oracle/) and the
seeded input generators (paper_2109_07358_amd/workloads.py, which holds none
of the sampler's arithmetic); nothing here loads or runs the HIP library.

Each fixture is the oracle's output for one workload, at the samples the
benchmark draws:

  c2_chain_L4096_N256.npz  disordered chain (lowest 256 eigenvectors of
                           hopping -1 with on-site energies uniform in
                           [-1, 1], seed 2), Philox seed 0x5EED, samples
                           0 .. 12287 (the first three S = 4096 calls of the
                           benchmark), all 256 steps: 3,145,728 draws.
  c3_complex_L16384_N512.npz
                           complex Gaussian-QR orbitals (seed 3), Philox
                           seed 1, 32 complete 512-step samples spread over
                           the S = 8192 call (both half-batches, several
                           column tiles).

Stored per fixture: the drawn sites (draw order), log|det U[x,:]|^2, every
draw whose oracle margin (relative distance of u*T to the nearer end of the
drawn site's CDF interval, Eq. (2)'s inverse-CDF draw) is below 1e-6 with
that margin, and a probe of U (a few full rows) so a test can check that its
input is the one the fixture was made from.

Usage: python tests/golden/make_golden.py [c2|c3|all] [--procs P]
"""
import argparse
import multiprocessing as mp
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

NEAR = 1e-6          # margins below this are stored
PROBE_ROWS = 8

_U = None


def _work(args):
    from threadpoolctl import threadpool_limits
    from oracle import sampler
    seed, s = args
    with threadpool_limits(1):
        r = sampler.sample_one(_U, seed, s)
    return s, np.array(r["x"]), r["logdet"], np.array(r["margin"])


def make(name, U, seed, samples, workload, procs):
    global _U
    _U = U
    L, N = U.shape
    n = len(samples)
    X = np.zeros((n, N), dtype=np.uint16)
    ld = np.zeros(n)
    mins = np.zeros(n)
    near = []
    row_of = {int(s): i for i, s in enumerate(samples)}
    t0 = time.time()
    done = 0
    with mp.get_context("fork").Pool(procs) as pool:
        for s, x, l, m in pool.imap_unordered(_work, [(seed, int(s)) for s in samples],
                                              chunksize=4):
            i = row_of[s]
            X[i] = x
            ld[i] = l
            mins[i] = m.min()
            for k in np.nonzero(m < NEAR)[0]:
                near.append((i, int(k), float(m[k])))
            done += 1
            if done % 256 == 0 or done == n:
                print("%s: %d/%d samples, %.0f s" % (name, done, n, time.time() - t0),
                      flush=True)
    near.sort()
    rows = np.linspace(0, L - 1, PROBE_ROWS).astype(np.int64)
    out = os.path.join(HERE, name + ".npz")
    np.savez_compressed(
        out, sites=X, logdet=ld, min_margin=mins, samples=np.asarray(samples, dtype=np.int64),
        near_idx=np.array([(i, k) for i, k, _ in near], dtype=np.int64).reshape(-1, 2),
        near_margin=np.array([m for _, _, m in near], dtype=np.float64),
        probe_rows=rows, probe=U[rows], seed=np.uint64(seed), L=L, N=N,
        workload=np.array(workload))
    print("wrote", out, os.path.getsize(out), "bytes;", len(near), "draws with margin <",
          NEAR, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("which", nargs="?", default="all", choices=["c2", "c3", "all"])
    ap.add_argument("--procs", type=int, default=os.cpu_count() or 1)
    a = ap.parse_args()
    from paper_2109_07358_amd import workloads
    if a.which in ("c3", "all"):
        U = workloads.gaussian_qr(16384, 512, 3, complex_=True)
        samples = np.concatenate([np.arange(0, 8), np.arange(2044, 2052),
                                  np.arange(4092, 4100), np.arange(8184, 8192)])
        make("c3_complex_L16384_N512", U, 1, samples,
             "complex gaussian_qr L=16384 N=512 seed=3; Philox seed 1; 32 complete samples "
             "of the S=8192 call", a.procs)
    if a.which in ("c2", "all"):
        U = workloads.anderson_chain(4096, 256, 2.0, 2)
        make("c2_chain_L4096_N256", U, 0x5EED, np.arange(3 * 4096),
             "anderson_chain L=4096 N=256 W=2 seed=2; Philox seed 0x5EED; samples 0..12287 "
             "(three S=4096 calls)", a.procs)


if __name__ == "__main__":
    main()
