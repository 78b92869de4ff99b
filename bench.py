#!/usr/bin/env python3
"""Benchmark of the FFS hot path on one MI355X.

Workload (default): the disordered 1D chain, L=4096 sites, N=256 particles
(lowest-N eigenvectors of hopping -1 with on-site energies uniform in
[-1, 1], seed 2), S=4096 samples per step.  A "step" is one ffs_sample call
drawing S complete configurations through the batched path: per particle
k = 1..N the float64 factor update/solve, the all-site FP32-MFMA weight
contraction, the inverse-CDF draw with its guard, and the float64 redraw of
guarded draws.  Inputs (U, working memory) are resident in HBM before the
timed region.

Reported: samples/s (value), ms per step, p50/p99 step latency, the plain
one-sample-per-launch path on the same U (speedup), useful (LN^2 + N^3 per
sample, the paper's count) and executed TFLOP/s, the dominant kernel's
roofline from HIP events bound to each of its launches inside the timed
region (next to each launch's own span on the device's steady clock),
guard statistics, the CPU oracle on a bounded sample, and the
complex L=16384, N=512, S=8192 contraction's fraction of FP32 MFMA peak.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3   # MI355X dense FP32 matrix
PEAK_HBM_GBS = 8000.0      # MI355X HBM3E

# HBM bytes per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE passes over one
# L=4096 N=256 call (2048-sample launches, the benchmark's 64x64k16 tile),
# each counter scaled by what it reads for a 1 GiB device copy (FETCH_SIZE
# x2.000, WRITE_SIZE x1.000).  A
# figure is only reported while the kernel's sources still hash to the
# values the counters were taken with.
MEASURED_TRAFFIC = {
    "weights": {"tiles": {"64x64k16": 67205703.1},
                "sources": {"k_weights.hip": "ae5df5c12c3af4b0",
                            "weights_common.h": "a00453495784e017"}},
    "factor": {"bytes_per_launch": 152197405.0,
               "sources": {"k_batched.hip": "8763213b49af59ef",
                           "factor_blk.h": "60edc12fbab8b266",
                           "draw.h": "9117d97cc061ed4e"}},
}


def measured_traffic(kind, tile=None):
    import hashlib
    rec = MEASURED_TRAFFIC[kind]
    if "tiles" in rec:
        if tile not in rec["tiles"]:
            return None
    elif tile is not None and rec.get("tile") not in (None, tile):
        return None
    for f, h in rec["sources"].items():
        path = os.path.join(ROOT, "paper_2109_07358_amd", "csrc", f)
        with open(path, "rb") as fh:
            if hashlib.sha256(fh.read()).hexdigest()[:16] != h:
                return None
    return rec["tiles"][tile] if "tiles" in rec else rec["bytes_per_launch"]


def _oracle_worker(args):
    from threadpoolctl import threadpool_limits
    from oracle import sampler
    U, seed, s = args
    with threadpool_limits(1):
        sampler.sample_one(U, seed, s)
    return s


def cpu_baseline(U, seed, n_samples, cores, first=0):
    """The oracle as it stands, timed on the host over a bounded sample:
    `cores` processes (1 = in this process) with one BLAS thread each."""
    import multiprocessing as mp
    work = [(U, seed, s) for s in range(first, first + n_samples)]
    t0 = time.perf_counter()
    if cores == 1:
        for a in work:
            _oracle_worker(a)
    else:
        with mp.get_context("fork").Pool(cores) as pool:
            list(pool.imap_unordered(_oracle_worker, work))
    dt = time.perf_counter() - t0
    return n_samples / dt, dt


def host_info():
    """Host cores (all, and usable by this process) and CPU model."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"nproc": os.cpu_count(), "usable_cpus": usable, "cpu_model": model}


def factor_bytes(L, N, S, es, n_steps, BB=16):
    """Algorithmic HBM bytes of all factor launches of one call.

    Regular launch at step t (block start t0): reads the t0 x 16 block
    solution E twice (update, solve), writes one row of G, beta and Gamma and
    the drawn row's entries in later blocks' columns (N - t0 - 16 words).
    Block-closing launch: reads the t0 x t0 inverse factors twice (one
    16-right-hand-side product per triangle in each direction) and ~10 t0 x 16
    panels."""
    tot = 0
    for t in range(-1, n_steps):
        tt = max(t, 0)
        t0 = (tt // BB) * BB
        tot += S * (2 * t0 * BB * es + (t0 + tt + 1) * es + 8 * N
                    + max(0, N - t0 - BB) * es)
        if t >= 0 and t % BB == BB - 1 and t + 1 < n_steps:
            tot += S * (2 * t0 * t0 * es + 10 * t0 * BB * es)
    return tot


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--samples", type=int, default=4096)
    ap.add_argument("--plain-samples", type=int, default=24)
    ap.add_argument("--cpu-samples", type=int, default=24)
    ap.add_argument("--cpu-samples-1", type=int, default=8,
                    help="samples for the one-process oracle leg")
    ap.add_argument("--shadow-complex", type=int, default=0, metavar="CALLS",
                    help="compare every draw of CALLS complex L=16384 N=512 calls (S=2048) "
                         "with the same calls drawn entirely from float64 weights")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-c3", action="store_true")
    ap.add_argument("--tile", default=None, metavar="SITESxCOLS[kKC]",
                    help="contraction tile (e.g. 128x128, 64x64k16) or 'auto' for the pipeline "
                         "autotuner; default: the measured best, 64x64k16 for the two-stream "
                         "chain call, 128x128k16 for one stream and the complex contraction")
    ap.add_argument("--timing-stride", type=int, default=7,
                    help="time one contraction launch in this many inside the timed region")
    ap.add_argument("--one-stream", action="store_true",
                    help="run each chain call as one launch per step on one stream "
                         "(no half-batch overlap): the per-kernel profile of the step")
    ap.add_argument("--serving", action="store_true",
                    help="run the serving mix (Poisson arrivals of mixed L, N) "
                         "instead of the chain benchmark")
    ap.add_argument("--dpp", action="store_true",
                    help="run the DPP workload (L=20000 items, d=256 eigenvectors, "
                         "fixed-size eigen-subsets k=10/20/50, FP32 vs split-BF16)")
    ap.add_argument("--mh", action="store_true",
                    help="Metropolis conditional update (SI S-7) vs the exact path at L=65536")
    ap.add_argument("--shadow", type=int, default=0, metavar="CALLS",
                    help="compare every draw of CALLS chain calls with the plain float64 path")
    ap.add_argument("--jastrow", action="store_true",
                    help="Slater-Jastrow reweighting of chain samples of both spins")
    ap.add_argument("--grouped", action="store_true",
                    help="16 and 64 mixed requests (L <= 16384, N <= 256): separate calls vs "
                         "the request server vs one grouped run (eager and hipGraph)")
    ap.add_argument("--complex-full", action="store_true",
                    help="complete samples of the complex L=16384, N=512 workload "
                         "(S=8192 per call): FP32 and split-BF16 at two guard deltas")
    ap.add_argument("--rate", type=float, default=2000.0)
    ap.add_argument("--duration", type=float, default=0.25)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--serve-mode", default="grouped", choices=["grouped", "streams"])
    ap.add_argument("--capacity", type=int, default=128)
    ap.add_argument("--ticks", type=int, default=8)
    ap.add_argument("--sustained-rates", default="25,50",
                    help="comma-separated request rates for 4 s runs")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device-to-device five times (the "
                         "known-size kernel that scales HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the sampler shards over "
              "samples with no exchange, so N>1 is not run here.", file=sys.stderr)
        sys.exit(2)

    if args.copy_probe:
        import torch
        n = args.copy_probe << 18
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": 4 * n}), flush=True)
        return

    if args.serving:
        return serving_main(args)
    if args.dpp:
        return dpp_main(args)
    if args.mh:
        return mh_main(args)
    if args.shadow:
        return shadow_main(args)
    if args.shadow_complex:
        return shadow_complex_main(args)
    if args.jastrow:
        return jastrow_main(args)
    if args.complex_full:
        return complex_full_main(args)
    if args.grouped:
        return grouped_main(args)

    import numpy as np
    from paper_2109_07358_amd import workloads
    L, N, S, seed = 4096, 256, args.samples, 0x5EED
    U = workloads.anderson_chain(L, N, 2.0, 2)

    cpu = None
    if not args.no_cpu:
        # a one-GPU job gets a 16-CPU share of the host, whatever nproc shows
        hi = host_info()
        cores = max(1, min(16, hi["usable_cpus"] or 1))
        rate1, dt1 = cpu_baseline(U, seed, args.cpu_samples_1, 1, first=10 ** 6)
        rate, dt = cpu_baseline(U, seed, args.cpu_samples, cores)
        cpu = {"value": rate, "unit": "samples/s", "cores": cores,
               "kind": "oracle",
               "sample": "%d samples of the L=4096 N=256 chain, %d processes "
                         "x 1 BLAS thread, %.1f s wall" % (args.cpu_samples, cores, dt),
               "one_process": {"value": rate1, "unit": "samples/s", "cores": 1,
                               "sample": "%d samples, 1 process x 1 BLAS thread, %.1f s wall"
                                         % (args.cpu_samples_1, dt1)},
               "useful_gflops": (L * N * N + N ** 3) * rate / 1e9,
               "host": hi,
               "pool_note": "pool capped at 16 processes: the CPU share of one GPU's job"}

    import torch
    from paper_2109_07358_amd import ffs
    torch.cuda.set_device(0)
    ffs.load()
    plan = ffs.ffs_plan(U, overlap=not args.one_stream)
    if args.tile == "auto":
        tile = ffs.ffs_autotune(plan, S, pipeline=True)  # contraction tile, timed in the pipeline
    else:
        tile = args.tile or ("128x128k16" if args.one_stream else "64x64k16")
        ffs.ffs_set_tile(plan, S, tile)
    x = torch.empty((S, N), dtype=torch.int32, device="cuda")
    for w in range(args.warmup):
        ffs.ffs_sample(plan, seed, 10 ** 9 + w * S, S, x_out=x)
    torch.cuda.synchronize()
    ffs.ffs_kernel_times(plan)
    ffs.ffs_kernel_spans(plan)
    # inside the timed region only the contraction (the dominant kernel) is
    # timed, and only one launch in --timing-stride (an odd stride samples
    # both half-batches and every step phase): each event pair leaves the
    # GPU idle for ~10 us around its launch
    ffs.ffs_set_timing_classes(plan, ["weights"])
    ffs.ffs_set_timing_stride(plan, args.timing_stride)

    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs[0].record()
    for k in range(args.steps):
        ffs.ffs_sample(plan, seed, k * S, S, x_out=x)
        evs[k + 1].record()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    st = ffs.ffs_check(plan)
    ktimed = ffs.ffs_kernel_times(plan)
    span_ms, span_n = ffs.ffs_kernel_spans(plan)
    step_ms = [evs[k].elapsed_time(evs[k + 1]) for k in range(args.steps)]
    value = args.steps * S / elapsed
    ms_per_step = elapsed * 1e3 / args.steps
    # per-class breakdown from one more call with every launch timed
    ffs.ffs_set_timing_stride(plan, 1)
    ffs.ffs_set_timing(plan, True)
    ffs.ffs_sample(plan, seed, 2 * 10 ** 9, S, x_out=x)
    torch.cuda.synchronize()
    ktimes = ffs.ffs_kernel_times(plan)
    ffs.ffs_set_timing(plan, False)

    # plain path, same U, one launch per sample
    pplan = ffs.ffs_plan(U, path="plain")
    xp = torch.empty((1, N), dtype=torch.int32, device="cuda")
    for w in range(2):
        ffs.ffs_sample(pplan, seed, w, 1, x_out=xp)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for s in range(args.plain_samples):
        ffs.ffs_sample(pplan, seed, s, 1, x_out=xp)
    torch.cuda.synchronize()
    plain_rate = args.plain_samples / (time.perf_counter() - t1)

    useful = (L * N * N + N ** 3) * value / 1e12
    executed_gemm = 2.0 * L * N * S * N * args.steps / elapsed / 1e12
    es = 8
    # dominant kernel: the contraction (largest single kernel by device time).
    # Its algorithmic work is the method's: 2 L k flops per sample at step k
    # (the 2Lk term of the cost count after Eq. (3)), summed over the call's
    # steps: L N (N + 1) S.  The kernel runs dense over the N columns
    # (2 L N S per launch), which is reported as the executed rate.
    # Per launch: the call's work over its contraction launches (N per
    # half-batch, counted in the every-launch breakdown call), against the
    # mean duration of the sampled launches.
    launches_per_call = ktimes["weights"][1]
    gemm_flops = 2.0 * L * N * S * N / launches_per_call
    method_flops = float(L) * N * (N + 1) * S / launches_per_call
    ms_launch = ktimed["weights"][0] / (ktimed["weights"][1] or 1)
    achieved = method_flops / (ms_launch * 1e-3) / 1e12
    executed = gemm_flops / (ms_launch * 1e-3) / 1e12
    roof = {"kernel": "weights_kernel (FP32 MFMA contraction)",
            "bound": "mfma", "achieved": achieved, "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS,
            # counters were taken on the two-stream call's 2048-sample launches
            "traffic": None if args.one_stream else measured_traffic("weights", tile),
            "traffic_unit": "HBM bytes per launch (rocprofv3, scaled)",
            "work": "method: sum_k 2 L k flops per sample (L N (N+1) per call and sample)",
            "executed_tflops": executed, "executed_frac": executed / PEAK_FP32_TFLOPS,
            "ms_per_launch": ms_launch,
            "launches": ktimed["weights"][1],
            "launches_in_timed_region": launches_per_call * args.steps,
            "method_flops_per_launch": method_flops,
            "timing": "HIP events bound to the dispatch of one launch in %d"
                      % args.timing_stride,
            "kernel_span_ms_per_launch": span_ms / (span_n or 1),
            "kernel_span_note": "each launch's own span on the device steady clock (first "
                                "workgroup start to last workgroup end): leaves out the wait "
                                "for CUs held by the other half-batch's kernels"}
    kernel_ms = {k: round(v[0], 3) for k, v in ktimes.items()}
    contraction_tflops = executed
    f_ms = ktimes["factor"][0] + ktimes["factor_block"][0]
    factor_gbs = factor_bytes(L, N, S, es, N) / (f_ms * 1e-3) / 1e9 if f_ms else None

    c3 = None
    if not args.no_c3:
        del plan
        torch.cuda.empty_cache()
        c3 = c3_contraction(ffs, torch, args.tile)

    out = {
        "metric": "samples/s + achieved TFLOP/s vs plain path at L=4096,N=256; p50/p99 latency",
        "value": value, "unit": "samples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "anderson_chain L=4096 N=256 W=2 seed=2; S=4096 "
                               "samples per step; FP32 bulk, FP64 factors",
                   "global_batch": S, "parallelism": "single GPU",
                   "streams": 1 if args.one_stream else 2},
        "p50_step_ms": float(np.percentile(step_ms, 50)),
        "p99_step_ms": float(np.percentile(step_ms, 99)),
        "plain_samples_per_s": plain_rate,
        "speedup_vs_plain": value / plain_rate,
        "useful_tflops": useful,
        "executed_contraction_tflops": executed_gemm,
        "kernel_ms_per_step": kernel_ms,
        "kernel_ms_note": "one extra call with every launch timed; factor_block = the "
                          "factor launches that close a 16-step block",
        "contraction_kernel_tflops": contraction_tflops,
        "factor_kernel_gbs": factor_gbs,
        "guard": {"draws": st["draws"], "flagged": st["flagged"],
                  "changed": st["changed"]},
        "contraction_tile": tile,
        "roofline": roof,
        "cpu_baseline": cpu,
        "c3_contraction": c3,
    }
    print(json.dumps(out), flush=True)


def c3_contraction(ffs, torch, tile_arg=None):
    """FP32-MFMA contraction at the complex L=16384, N=512, S=8192 shape.

    Runs the first 16 steps (ffs_marginal): the contraction's shape does not
    depend on the step, so its per-launch time is that of a full run."""
    from paper_2109_07358_amd import workloads
    L, N, S = 16384, 512, 8192
    U = workloads.gaussian_qr(L, N, 3, complex_=True)
    plan = ffs.ffs_plan(U, max_batch=S, overlap=False)  # one launch per step, alone on the stream
    if tile_arg == "auto":
        tile = ffs.ffs_autotune(plan, S)
    else:
        # the complex contraction's tiles have 128 GEMM columns
        ok = tile_arg and ffs.parse_tile(tile_arg)[1] == 128
        tile = tile_arg if ok else "128x128k16"
        ffs.ffs_set_tile(plan, S, tile)
    keep = 16
    ffs.ffs_marginal(plan, keep, 1, 0, S)
    torch.cuda.synchronize()
    ffs.ffs_kernel_times(plan)
    ffs.ffs_set_timing(plan, True)
    ffs.ffs_marginal(plan, keep, 1, S, S)
    torch.cuda.synchronize()
    kt = ffs.ffs_kernel_times(plan)
    ms, n = kt["weights"]
    assert n == keep, n
    # a dense complex product over N counts 8 L N S flops per launch (a
    # complex multiply-add as 8 real flops); the kernel's Gauss form runs
    # three real products, 6 L N S, on the matrix cores
    tf = 8.0 * L * N * S * n / (ms * 1e-3) / 1e12
    te = 6.0 * L * N * S * n / (ms * 1e-3) / 1e12
    # the launch is dense over N, so its duration does not depend on the
    # step: over a complete 512-step call the method's work (8 L k flops per
    # sample at step k) is (N + 1) / (2 N) of the dense product
    tm = tf * (N + 1) / (2.0 * N)
    return {"workload": "complex gaussian_qr L=16384 N=512 S=8192, first %d steps" % keep,
            "tile": tile, "ms_per_launch": ms / n,
            "dense_complex_tflops": tf, "dense_complex_frac_of_fp32_peak": tf / PEAK_FP32_TFLOPS,
            "executed_tflops": te, "executed_frac_of_fp32_peak": te / PEAK_FP32_TFLOPS,
            "method_tflops_full_call": tm, "method_frac_of_fp32_peak": tm / PEAK_FP32_TFLOPS}


def grouped_main(args):
    """Many small instances at once: the same mixed requests (Gaussian-QR U for
    each (L, N) in {1024, 4096, 16384} x {16, 64, 256}, 1-256 samples, seeded)
    run as separate ffs_marginal calls, through the request server (4 slots),
    and as one grouped run (ffs_sample_group), eager and captured; every way
    must give the same configurations."""
    import numpy as np
    import torch
    from paper_2109_07358_amd import ffs, workloads
    torch.cuda.set_device(0)
    ffs.load()
    rng = np.random.default_rng(3)
    pairs = [(L, N) for L in (1024, 4096, 16384) for N in (16, 64, 256)]
    pool = {p: ffs.ffs_plan(workloads.gaussian_qr(p[0], p[1], 200 + k)) for k, p in enumerate(pairs)}
    runs = []
    for n_req in (16, 64):
        spec = []
        for _ in range(n_req):
            L, N = pairs[int(rng.integers(0, len(pairs)))]
            spec.append((L, N, int(rng.integers(1, 257)), int(rng.integers(0, 2 ** 40))))
        outs = [torch.empty((n, N), dtype=torch.int32, device="cuda") for (L, N, n, s) in spec]
        samples = sum(n for (_, _, n, _) in spec)

        def separate():
            for (L, N, n, s), x in zip(spec, outs):
                ffs.ffs_marginal(pool[(L, N)], N, s, 0, n, x_out=x)

        def grouped(graph):
            ffs.ffs_sample_group([{"plan": pool[(L, N)], "n_keep": N, "seed": s, "first_sample": 0,
                                   "n_samples": n, "x_out": x}
                                  for (L, N, n, s), x in zip(spec, outs)], graph=graph)

        def server():
            sv = ffs.Server(slots=4)
            ts = [sv.submit(pool[(L, N)], N, s, 0, n, x) for (L, N, n, s), x in zip(spec, outs)]
            for t in ts:
                sv.poll(t, -1)
            sv.close()

        ref = None
        for name, fn in [("separate", separate), ("server", server),
                         ("grouped", lambda: grouped(False)), ("grouped_graph", lambda: grouped(True))]:
            fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(3):
                fn()
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / 3
            cur = [x.cpu().numpy().copy() for x in outs]
            ref = cur if ref is None else ref
            same = all(np.array_equal(a, b) for a, b in zip(ref, cur))
            runs.append({"requests": n_req, "samples": samples, "mode": name, "ms": dt * 1e3,
                         "samples_per_s": samples / dt, "same_as_separate": same})
            print("grouped: %d requests %s done" % (n_req, name), file=sys.stderr, flush=True)
    head = [r for r in runs if r["requests"] == 64 and r["mode"] == "grouped"][0]
    sep = [r for r in runs if r["requests"] == 64 and r["mode"] == "separate"][0]
    out = {"metric": "samples/s of 64 mixed requests in one grouped run", "value": head["samples_per_s"],
           "unit": "samples/s", "n_gpus": 1, "steps": 3, "warmup": 1, "higher_is_better": True,
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "16 and 64 requests, Gaussian-QR U per (L, N), L in {1024,4096,16384}, "
                                  "N in {16,64,256}, 1-256 samples each, seed 3"},
           "speedup_vs_separate": head["samples_per_s"] / sep["samples_per_s"], "runs": runs}
    print(json.dumps(out), flush=True)


def complex_full_main(args):
    """Complete samples (all N = 512 steps) of the complex Gaussian-QR workload,
    L = 16384, S = 8192 per call, for the FP32 and split-BF16 contractions with
    their default (adaptive) guard; the whole call is timed, and the drawn
    sites' frequencies are compared with the site marginals diag(U U^dagger)."""
    import torch
    from paper_2109_07358_amd import ffs, workloads
    torch.cuda.set_device(0)
    ffs.load()
    import numpy as np
    L, N, S = 16384, 512, 8192
    U = workloads.gaussian_qr(L, N, 3, complex_=True)
    # site marginals diag(U U^dagger) in float64, binned by 256 sites
    rho = (U.real ** 2 + U.imag ** 2).sum(axis=1)
    bins = L // 256
    rho_b = rho.reshape(bins, 256).sum(axis=1)

    def marginal_error(X):
        """Drawn-site frequencies against diag(U U^dagger): max |z| over sites
        with rho > 1e-3 and chi^2/dof of the 256-site bin counts."""
        n = X.shape[0]
        freq = np.bincount(X.ravel(), minlength=L) / n
        sd = np.sqrt(np.maximum(rho * (1 - rho), 1e-12) / n)
        ok = rho > 1e-3
        h = np.bincount(X.ravel() // 256, minlength=bins).astype(np.float64)
        exp = rho_b * n
        return {"max_abs_z_site": float(np.max(np.abs((freq - rho) / sd)[ok])),
                "max_abs_freq_minus_rho": float(np.max(np.abs(freq - rho))),
                "binned_chi2_per_dof": float(((h - exp) ** 2 / exp).sum() / (bins - 1)),
                "sum_freq": float(freq.sum())}

    runs = []
    for bulk in ("fp32", "split_bf16"):
        for delta in (None,):
            plan = ffs.ffs_plan(U, max_batch=S, bulk=bulk, guard_delta=delta)
            x = torch.empty((S, N), dtype=torch.int32, device="cuda")
            # warm-up: tiles, working memory, and the resolution mode the
            # plan settles on (a call that needs a replay turns deferred
            # resolution off for the next ones)
            ffs.ffs_sample(plan, 1, 10 ** 9, S, x_out=x)
            torch.cuda.synchronize()
            ffs.ffs_check(plan)
            t0 = time.perf_counter()
            ffs.ffs_sample(plan, 1, 0, S, x_out=x)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            st = ffs.ffs_check(plan)
            runs.append({"bulk": bulk, "guard": "default (adaptive)" if delta is None else delta,
                         "s_per_call": dt, "samples_per_s": S / dt,
                         "useful_tflops": 4.0 * (L * N * N + N ** 3) * S / dt / 1e12,
                         "guard_stats": st,
                         "marginals_vs_diag_UUdag": marginal_error(x.cpu().numpy())})
            print("complex-full: %s delta %s done" % (bulk, delta), file=sys.stderr, flush=True)
            del plan, x
            torch.cuda.empty_cache()
    head = runs[0]
    out = {"metric": "complex samples/s, complete samples", "value": head["samples_per_s"],
           "unit": "samples/s", "n_gpus": 1, "steps": 1, "warmup": 1, "higher_is_better": True,
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "complex gaussian_qr L=16384 N=512 seed=3; S=8192 complete samples "
                                  "per call; complex64 bulk, complex128 factors"},
           "runs": runs}
    print(json.dumps(out), flush=True)


def dpp_main(args):
    """DPP sampling: device front end (dual eigendecomposition, eigenvector
    selection) and the projection stage (per-sample eigenvector subsets)."""
    import numpy as np
    import torch
    from paper_2109_07358_amd import ffs, workloads
    torch.cuda.set_device(0)
    ffs.load()
    L, d, S = 20000, 256, args.samples
    B = torch.from_numpy(workloads.dpp_features(L, d, 4)).cuda()
    ffs.ffs_dpp_eig(B)  # warm-up (allocator, code objects)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lam, V, _, sweeps = ffs.ffs_dpp_eig(B)
    eig_ms = (time.perf_counter() - t0) * 1e3
    print("dpp: eigendecomposition %.1f ms, %d sweeps" % (eig_ms, sweeps), file=sys.stderr,
          flush=True)
    configs = [("fp32", None), ("split_bf16", None), ("split_bf16", 2.0 ** -20)]
    plans = {c: ffs.ffs_plan(V, bulk=c[0], guard_delta=c[1]) for c in configs}
    runs = []
    n_calls = args.warmup + args.steps
    for k in (10, 20, 50):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cols = ffs.ffs_kdpp_subsets(lam, k, k, 0, S * n_calls)
        torch.cuda.synchronize()
        sel_ms = (time.perf_counter() - t0) * 1e3
        x = torch.empty((S, k), dtype=torch.int32, device="cuda")
        ref = None  # FP32 draws of the timed calls
        for (bulk, delta), plan in plans.items():
            xs = []
            for c in range(args.warmup):
                ffs.ffs_sample_subsets(plan, cols[c * S:(c + 1) * S], 4, c * S, x_out=x)
            torch.cuda.synchronize()
            ffs.ffs_kernel_times(plan)
            ffs.ffs_set_timing_classes(plan, ["weights"])
            t0 = time.perf_counter()
            flagged = changed = 0
            for c in range(args.warmup, n_calls):
                ffs.ffs_sample_subsets(plan, cols[c * S:(c + 1) * S], 4, c * S, x_out=x)
                st = ffs.ffs_check(plan)
                flagged += st["flagged"]
                changed += st["changed"]
                xs.append(x.clone())
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            xs = torch.cat(xs).cpu().numpy()
            if ref is None:
                ref = xs
            differ = int((xs != ref).any(axis=1).sum())
            kt = ffs.ffs_kernel_times(plan)
            ffs.ffs_set_timing(plan, False)
            ms_w, n_w = kt["weights"]
            flops = 2.0 * L * d * S * n_w
            runs.append({"k": k, "bulk": bulk,
                         "guard_delta": delta if delta is not None else "default",
                         "samples_per_s": S * args.steps / dt,
                         "ms_per_call": dt * 1e3 / args.steps,
                         "selection_ms_per_call": sel_ms / n_calls,
                         "contraction_fp32_equiv_tflops": flops / (ms_w * 1e-3) / 1e12,
                         "guard": {"draws": S * k * args.steps, "flagged": flagged,
                                   "changed": changed},
                         "samples_differing_from_fp32": differ})
            print("dpp: k=%d %s delta %s done" % (k, bulk, delta), file=sys.stderr, flush=True)
    # the paper's rule: eigenvector j kept with probability lambda_j/(lambda_j+1),
    # sample sizes vary; quality scaled so that about 20 of the 256 are kept
    lam_r = lam * 0.0004
    S_r = S // 4
    plan = plans[("fp32", None)]
    x = None
    for c in range(n_calls):
        if c == args.warmup:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
        cols, sizes = ffs.ffs_dpp_subsets(lam_r, 8, c * S_r, S_r)
        x, _ = ffs.ffs_sample_dpp(plan, cols, sizes, 9, c * S_r)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    sz = sizes.cpu().numpy()
    st = ffs.ffs_check(plan)
    runs.append({"rule": "lambda/(lambda+1)", "lambda_scale": 0.0004, "bulk": "fp32",
                 "samples_per_s": S_r * args.steps / dt, "ms_per_call": dt * 1e3 / args.steps,
                 "size_mean": float(sz.mean()), "size_min": int(sz.min()),
                 "size_max": int(sz.max()), "guard_last_call": st})
    print("dpp: lambda/(lambda+1) rule done", file=sys.stderr, flush=True)
    head = [r for r in runs if r.get("k") == 20 and r["bulk"] == "fp32"][0]
    out = {"metric": "DPP samples/s (projection stage, per-sample eigen-subsets)",
           "value": head["samples_per_s"], "unit": "samples/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "higher_is_better": True,
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "DPP: L=20000 items, d=256 row-normalised Gaussian features, "
                                  "LogNormal(0,0.5) quality; device dual eigendecomposition; "
                                  "k-DPP eigen-subsets k=10/20/50 selected on the device; "
                                  "S=%d samples per call" % S},
           "front_end": {"eig_ms": eig_ms, "jacobi_sweeps": sweeps,
                         "lambda_min": float(lam[0]), "lambda_max": float(lam[-1])},
           "runs": runs}
    print(json.dumps(out), flush=True)


def mh_main(args):
    """Metropolis conditional update (SI S-7) against the exact batched path
    at large L: throughput and a binned-density check of both, on localised
    (disordered chain) and delocalised (Gaussian) orbitals."""
    import numpy as np
    import torch
    from paper_2109_07358_amd import ffs, workloads
    torch.cuda.set_device(0)
    ffs.load()
    L, N, S = 65536, 256, 1024
    bins = 256
    runs = []
    for name, U in (("anderson_chain W=2", workloads.anderson_chain(L, N, 2.0, 2)),
                    ("gaussian_qr", workloads.gaussian_qr(L, N, 6))):
        rho_b = (U * U).sum(1).reshape(bins, -1).sum(1)
        plan = ffs.ffs_plan(U)

        def density_check(X):
            h = np.bincount(X.ravel() // (L // bins), minlength=bins).astype(np.float64)
            exp = rho_b * X.shape[0]
            keep = exp > 5
            return float(((h - exp) ** 2 / exp)[keep].sum() / max(1, keep.sum() - 1))

        x = torch.empty((S, N), dtype=torch.int32, device="cuda")
        ffs.ffs_sample(plan, 1, 0, S, x_out=x)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Xs = []
        for c in range(args.steps):
            ffs.ffs_sample(plan, 1, (c + 1) * S, S, x_out=x)
            Xs.append(x.cpu().numpy())
        dt = time.perf_counter() - t0
        runs.append({"orbitals": name, "path": "exact (all-site contraction)",
                     "samples_per_s": S * args.steps / dt, "ms_per_call": dt * 1e3 / args.steps,
                     "binned_density_chi2_per_dof": density_check(np.concatenate(Xs))})
        print("mh: %s exact path done" % name, file=sys.stderr, flush=True)
        for m_cond, radius in ((32, 16), (128, 16), (128, 0)):
            ffs.ffs_sample_mh(plan, m_cond, radius, 2, 0, S, x_out=x)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            Xs, acc = [], 0
            for c in range(args.steps):
                _, _, a = ffs.ffs_sample_mh(plan, m_cond, radius, 2, (c + 1) * S, S, x_out=x,
                                            accepted=True)
                acc += a
                Xs.append(x.cpu().numpy())
            dt = time.perf_counter() - t0
            runs.append({"orbitals": name, "path": "metropolis", "m_cond": m_cond,
                         "radius": radius, "samples_per_s": S * args.steps / dt,
                         "ms_per_call": dt * 1e3 / args.steps,
                         "acceptance": acc / (S * N * m_cond * args.steps),
                         "binned_density_chi2_per_dof": density_check(np.concatenate(Xs))})
            print("mh: %s m_cond=%d radius=%d done" % (name, m_cond, radius), file=sys.stderr,
                  flush=True)
        del plan
    head = [r for r in runs if r["orbitals"] == "gaussian_qr" and r.get("m_cond") == 128
            and r.get("radius") == 0][0]
    out = {"metric": "samples/s, Metropolis conditional update vs exact path at L=65536",
           "value": head["samples_per_s"], "unit": "samples/s", "n_gpus": 1,
           "steps": args.steps, "warmup": 1, "higher_is_better": True, "vs_baseline": None,
           "dtype": "f64", "data": "synthetic",
           "config": {"workload": "L=65536 N=256 (disordered chain W=2; Gaussian QR); S=%d "
                                  "samples per call; density check: chi2/dof of 256-site bin "
                                  "counts against diag(U U^T)" % S},
           "runs": runs}
    print(json.dumps(out), flush=True)


def shadow_main(args):
    """Draw-level agreement at scale: the batched FP32 path (with its float64
    guard) against the plain float64 path on the same samples of the chain
    workload, every draw compared."""
    import numpy as np
    import torch
    from paper_2109_07358_amd import ffs, workloads
    torch.cuda.set_device(0)
    ffs.load()
    L, N, S, seed = 4096, 256, 4096, 0x5EED
    n_calls = args.shadow
    U = workloads.anderson_chain(L, N, 2.0, 2)
    plan = ffs.ffs_plan(U)
    pplan = ffs.ffs_plan(U, path="plain", bulk="fp64")
    streams = [torch.cuda.Stream() for _ in range(16)]
    mism_draws = mism_samples = flagged = changed = 0
    t_plain = 0.0
    for c in range(n_calls):
        first = c * S
        xb, _ = ffs.ffs_sample(plan, seed, first, S)
        torch.cuda.synchronize()
        st = ffs.ffs_check(plan)
        flagged += st["flagged"]
        changed += st["changed"]
        xp = torch.empty((S, N), dtype=torch.int32, device="cuda")
        per = S // len(streams)
        t0 = time.perf_counter()
        for k, sk in enumerate(streams):
            ffs.ffs_sample(pplan, seed, first + k * per, per, x_out=xp[k * per:(k + 1) * per],
                           stream=sk)
        torch.cuda.synchronize()
        t_plain += time.perf_counter() - t0
        d = (xb != xp).cpu().numpy()
        mism_draws += int(d.sum())
        mism_samples += int(d.any(axis=1).sum())
        print("shadow: call %d compared (%d mismatched draws so far)" % (c, mism_draws),
              file=sys.stderr, flush=True)
    draws = n_calls * S * N
    out = {"metric": "draw mismatches, batched FP32 + guard vs plain float64 path",
           "value": mism_draws, "unit": "draws", "n_gpus": 1, "steps": n_calls, "warmup": 0,
           "higher_is_better": False, "vs_baseline": None, "dtype": "f32 vs f64",
           "data": "synthetic",
           "config": {"workload": "anderson_chain L=4096 N=256 W=2 seed=2; %d calls of S=4096 "
                                  "samples, every draw compared" % n_calls},
           "draws_compared": draws, "mismatched_samples": mism_samples,
           "mismatch_rate_per_draw": mism_draws / draws,
           "rule_of_three_bound_if_zero": 3.0 / draws,
           "guard": {"flagged": flagged, "changed": changed},
           "plain_path_samples_per_s_16_streams": n_calls * S / t_plain}
    print(json.dumps(out), flush=True)


def shadow_complex_main(args):
    """Draw-level agreement at the complex L=16384, N=512 shape: the default
    batched FP32 path (adaptive guard) against the same calls with every
    draw taken from float64 weights (guard_delta = 1), every draw compared."""
    import numpy as np
    import torch
    from paper_2109_07358_amd import ffs, workloads
    torch.cuda.set_device(0)
    ffs.load()
    L, N, S, seed = 16384, 512, 2048, 1
    U = workloads.gaussian_qr(L, N, 3, complex_=True)
    runs = []
    for bulk in ("fp32", "split_bf16"):
        plan = ffs.ffs_plan(U, bulk=bulk)
        ref = ffs.ffs_plan(U, bulk=bulk, guard_delta=1.0)
        mism_draws = mism_samples = flagged = changed = 0
        t_def = 0.0
        for c in range(args.shadow_complex):
            t0 = time.perf_counter()
            xb, _ = ffs.ffs_sample(plan, seed, c * S, S)
            torch.cuda.synchronize()
            t_def += time.perf_counter() - t0
            st = ffs.ffs_check(plan)
            flagged += st["flagged"]
            changed += st["changed"]
            xr, _ = ffs.ffs_sample(ref, seed, c * S, S)
            torch.cuda.synchronize()
            d = (xb != xr).cpu().numpy()
            mism_draws += int(d.sum())
            mism_samples += int(d.any(axis=1).sum())
            print("shadow-complex: %s call %d compared (%d mismatched samples so far)"
                  % (bulk, c, mism_samples), file=sys.stderr, flush=True)
        draws = args.shadow_complex * S * N
        runs.append({"bulk": bulk, "draws_compared": draws, "mismatched_samples": mism_samples,
                     "mismatched_draws": mism_draws, "flagged": flagged,
                     "flag_rate": flagged / draws, "changed": changed,
                     "rule_of_three_bound_if_zero": 3.0 / draws,
                     "default_samples_per_s": args.shadow_complex * S / t_def})
        del plan, ref
        torch.cuda.empty_cache()
    out = {"metric": "draw mismatches, default guard vs all draws from float64 weights",
           "value": sum(r["mismatched_draws"] for r in runs), "unit": "draws", "n_gpus": 1,
           "steps": args.shadow_complex, "warmup": 0, "higher_is_better": False,
           "vs_baseline": None, "dtype": "f32 vs f64", "data": "synthetic",
           "config": {"workload": "complex gaussian_qr L=16384 N=512 seed=3; %d calls of "
                                  "S=2048 complete samples, every draw compared"
                                  % args.shadow_complex},
           "runs": runs}
    print(json.dumps(out), flush=True)


def jastrow_main(args):
    """Slater-Jastrow reweighting (SI S-5) of chain samples of both spins:
    Gutzwiller factor, and a density Jastrow with an L x L matrix."""
    import numpy as np
    import torch
    from paper_2109_07358_amd import ffs, workloads
    torch.cuda.set_device(0)
    ffs.load()
    L, N, S = 4096, 256, 4096
    U = workloads.anderson_chain(L, N, 2.0, 2)
    plan = ffs.ffs_plan(U)
    xu, _ = ffs.ffs_sample(plan, 11, 0, S)
    xd, _ = ffs.ffs_sample(plan, 22, 0, S)
    rng = np.random.default_rng(7)
    a = rng.standard_normal((L, L)) * 1e-3
    vmat = torch.from_numpy((a + a.T) / 2).cuda()
    runs = []
    for label, V, vm in (("gutzwiller V=2", 2.0, None), ("density jastrow v ~ N(0,1e-6)", 0.0, vmat)):
        ffs.ffs_jastrow_estimate(xu, xd, L, V, vmat=vm)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            _, dens, summ = ffs.ffs_jastrow_estimate(xu, xd, L, V, vmat=vm)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        runs.append({"jastrow": label, "ms_per_estimate": dt * 1e3,
                     "configurations_per_s": S / dt, "ess": summ["ess"],
                     "double_occupancy_J": summ["D_J"], "double_occupancy_0": summ["D_0"],
                     "density_sum": float(dens.sum().item())})
        print("jastrow: %s done" % label, file=sys.stderr, flush=True)
    out = {"metric": "Slater-Jastrow reweighted estimates per second", "value": runs[0]["configurations_per_s"],
           "unit": "configurations/s", "n_gpus": 1, "steps": args.steps, "warmup": 1,
           "higher_is_better": True, "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "anderson_chain L=4096 N=256 per spin, S=%d configurations "
                                  "(up and down drawn with seeds 11 and 22)" % S},
           "runs": runs}
    print(json.dumps(out), flush=True)


def serving_pool(ffs, Ls=(1024, 4096, 16384, 65536), Ns=(16, 64, 256, 1024)):
    """One resident plan per valid (L, N) pair (N <= L/4): Gaussian-QR U."""
    from paper_2109_07358_amd import workloads
    pool = {}
    k = 0
    for L in Ls:
        for N in Ns:
            if N <= L // 4:
                pool[(L, N)] = ffs.ffs_plan(workloads.gaussian_qr(L, N, 100 + k))
                k += 1
                print("pool: plan L=%d N=%d ready" % (L, N), file=sys.stderr, flush=True)
    return pool


def serving_run(ffs, torch, pool, rate, duration, slots, seed, mode="grouped",
                capacity=128, ticks=8):
    """Open-loop Poisson trace through an ffs server; latency from submission."""
    import numpy as np
    from paper_2109_07358_amd import workloads
    trace = workloads.poisson_trace(rate, duration, seed)
    outs = [torch.empty((r["n"], r["N"]), dtype=torch.int32, device="cuda") for r in trace]
    torch.cuda.synchronize()
    srv = ffs.Server(mode=mode, slots=slots, capacity=capacity, ticks=ticks)
    t0 = time.perf_counter()
    tickets, slip = [], []
    for r, x in zip(trace, outs):
        dt = r["t"] - (time.perf_counter() - t0)
        if dt > 0:
            time.sleep(dt)
        slip.append(time.perf_counter() - t0 - r["t"])
        tickets.append(srv.submit(pool[(r["L"], r["N"])], r["N"], r["seed"], 0, r["n"], x))
    infos = []
    for i, t in enumerate(tickets):
        infos.append(srv.poll(t, -1))
        if i % 200 == 199:
            print("serving: %d of %d requests done" % (i + 1, len(tickets)),
                  file=sys.stderr, flush=True)
    srv.close()
    assert all(i["status"] == 0 for i in infos)
    lat = np.array([i["t_done"] - i["t_submit"] for i in infos]) * 1e3
    svc = np.array([i["t_done"] - i["t_admit"] for i in infos]) * 1e3
    que = np.array([i["t_admit"] - i["t_submit"] for i in infos]) * 1e3
    span = max(i["t_done"] for i in infos) - min(i["t_submit"] for i in infos)
    samples = sum(r["n"] for r in trace)
    draws = sum(r["n"] * r["N"] for r in trace)
    flops = sum(2.0 * r["L"] * r["N"] ** 2 * r["n"] for r in trace)
    return {"rate_req_per_s": rate, "trace_s": duration, "requests": len(trace),
            "mode": mode, "slots": slots, "capacity": capacity, "ticks": ticks,
            "makespan_s": span, "samples_per_s": samples / span,
            "draws_per_s": draws / span,
            "executed_contraction_tflops": flops / span / 1e12,
            "latency_ms": {"p50": float(np.percentile(lat, 50)),
                           "p99": float(np.percentile(lat, 99))},
            "queue_ms": {"p50": float(np.percentile(que, 50)),
                         "p99": float(np.percentile(que, 99))},
            "service_ms": {"p50": float(np.percentile(svc, 50)),
                           "p99": float(np.percentile(svc, 99))},
            "max_submit_slip_ms": float(max(slip) * 1e3),
            "guard": {"draws": int(sum(i["draws"] for i in infos)),
                      "flagged": int(sum(i["flagged"] for i in infos)),
                      "changed": int(sum(i["changed"] for i in infos))}}


def serving_main(args):
    import torch
    from paper_2109_07358_amd import ffs
    torch.cuda.set_device(0)
    ffs.load()
    pool = serving_pool(ffs)
    # warm-up: one small request per plan (kernel loading, memory pool)
    srv = ffs.Server(mode=args.serve_mode, slots=args.slots, capacity=args.capacity,
                     ticks=args.ticks)
    xs = {k: torch.empty((2, k[1]), dtype=torch.int32, device="cuda") for k in pool}
    torch.cuda.synchronize()
    for t in [srv.submit(p, k[1], 1, 0, 2, xs[k]) for k, p in pool.items()]:
        srv.poll(t, -1)
    srv.close()
    kw = dict(mode=args.serve_mode, capacity=args.capacity, ticks=args.ticks)
    runs = [serving_run(ffs, torch, pool, args.rate, args.duration, args.slots, 5, **kw)]
    for r in [float(v) for v in args.sustained_rates.split(",") if v]:
        runs.append(serving_run(ffs, torch, pool, r, 4.0, args.slots, 6, **kw))
    head = runs[0]
    out = {"metric": "serving mix: samples/s with p50/p99 request latency",
           "value": head["samples_per_s"], "unit": "samples/s", "n_gpus": 1,
           "higher_is_better": True, "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": "serving mix: Poisson arrivals, L in {1024,4096,16384,65536}, "
                                  "N in {16,64,256,1024} with N <= L/4, 1-256 samples, "
                                  "Gaussian-QR U resident per (L, N)"},
           "p50_latency_ms": head["latency_ms"]["p50"],
           "p99_latency_ms": head["latency_ms"]["p99"],
           "runs": runs}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
