#!/usr/bin/env python3
"""Benchmark of the fast bilinear matrix product on one MI355X.

Default workload (``--workload square``): effective GFLOP/s = 2 n^3 / t of
the fast FP64 product (Strassen-Winograd, depth 2) at n = 8192, next to the
library's own classical FP64 MFMA GEMM, with inputs resident in HBM.  One
step is one whole product C = A B (pre-additions, grouped leaf GEMM with
fused post-additions, outer post-addition).

Other workloads, each printing one JSON line of the same shape:
  --workload batched    512 products, n log-uniform in [128, 2048] (multiples
                        of 64), one persistent launch per dtype (FP64, FP32),
                        (algorithm, depth) per size from the autotuner
  --workload serving    1000 requests, n log-uniform in [256, 8192], 70 % FP32,
                        Poisson arrivals at 0.5, 0.9 and 1.5 x the serial
                        service rate; p50/p99 latency and throughput

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload square]
                       [--n N] [--algo winograd] [--depth 2] [--no-cpu-baseline]

The `roofline` object reports the dominant kernel against its MI355X peak,
timed live with HIP events recorded on the launch stream.  The
`cpu_baseline` object times the CPU oracle on the host cores and is the only
place this script touches the oracle (also for the sampled error checks).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "effective GFLOP/s (2n^3/t) fast vs classical MFMA GEMM at stated rel. error"
FP64_MFMA_PEAK_TFLOPS = 78.6
HBM_PEAK_GBS = 8000.0
CSRC = os.path.join(ROOT, "paper_2312_12732_amd", "csrc")
KERNEL_SRCS = [os.path.join(CSRC, f) for f in ("kernels_gemm.hip", "gemm_tile.h", "gemm_common.h")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_gemm_f64.json")


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=8192)
    ap.add_argument("--algo", default="winograd")
    ap.add_argument("--depth", type=int, default=2)
    ap.add_argument("--cutoff", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", choices=("square", "batched", "serving"), default="square")
    ap.add_argument("--requests", type=int, default=1000, help="serving: requests per arrival rate")
    return ap.parse_args()


def kernel_sha() -> str:
    """Hash of the sources that define the grouped GEMM kernel."""
    h = hashlib.sha256()
    for path in KERNEL_SRCS:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_for(workload: str):
    """HBM bytes per GEMM launch from the committed rocprofv3 counter summary,
    if it was taken on the current kernel source for this workload."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sha") != kernel_sha() or t.get("workload") != workload:
        return None
    return t.get("hbm_bytes_per_launch")


def cpu_baseline(args, A_host, B_host, C_gpu_host):
    """Time the CPU oracle's fast product on the same workload (bounded to
    roughly 10-30 s) and check the GPU result on sampled rows."""
    import numpy as np

    import mf_inputs as mi
    from oracle import algebra as oa
    from oracle import matmul as om

    table = {"winograd": mi.WINOGRAD, "strassen": mi.STRASSEN_PAPER, "strassen1969": mi.STRASSEN_1969}[args.algo]
    U, V, W, conv = mi.as_float_tables(table)
    alg = oa.canonical(2, U, V, W, conv)
    cores = oracle_cores()
    n = args.n
    runs, elapsed = 0, 0.0
    while runs < 3 and elapsed < 10.0:
        t0 = time.perf_counter()
        om.fast_mm(A_host, B_host, alg, args.depth, args.cutoff)
        elapsed += time.perf_counter() - t0
        runs += 1
    gflops = runs * 2.0 * n ** 3 / elapsed / 1e9
    rows = np.sort(np.random.default_rng(5).choice(n, size=min(n, 64), replace=False))
    ref = om.rows_reference(A_host, B_host, rows)
    err = om.rel_fro_error(C_gpu_host[rows], ref)
    return ({"value": round(gflops, 2), "unit": "GFLOP/s", "cores": int(cores), "kind": "oracle",
             "sample": f"{runs} full oracle fast_mm run(s) of the same workload (n={n}, {args.algo}, "
                       f"depth {args.depth}), numpy/OpenBLAS float64, {elapsed:.1f} s"}, err)


def timer(torch, stream):
    """Mean device time per call of fn over `steps` calls (HIP events on the
    launch stream), after `warmup` untimed calls."""
    def timed(fn, steps, warmup):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record(stream)
        for _ in range(steps):
            fn()
        t1.record(stream)
        torch.cuda.synchronize()
        return t0.elapsed_time(t1) / steps
    return timed


def oracle_cores():
    try:
        from threadpoolctl import threadpool_info
        return int(max((p.get("num_threads", 1) for p in threadpool_info()), default=1))
    except Exception:  # noqa: BLE001
        return os.cpu_count() or 1


def run_square(args):
    import torch

    import mf_inputs as mi
    from paper_2312_12732_amd import mf

    dev = torch.device("cuda:0")
    n = args.n
    A_host = mi.uniform(n, 10)
    B_host = mi.uniform(n, 11)
    A = torch.from_numpy(A_host).to(dev)
    B = torch.from_numpy(B_host).to(dev)
    C = torch.empty_like(A)
    Cc = torch.empty_like(A)
    algo = mf.mf_algo_builtin(args.algo)
    stream = torch.cuda.current_stream()
    timed = timer(torch, stream)

    # classical MFMA GEMM of the library (context: the method's own baseline)
    classical_ms = timed(lambda: mf.mf_classical_mm(A, B, Cc), max(3, args.steps // 2), 2)

    # fast product: warm-up, then the timed region with per-phase events
    for _ in range(args.warmup):
        mf.mf_fastmm(algo, args.depth, args.cutoff, A, B, C)
    torch.cuda.synchronize()
    mf.mf_phase_timing_read()
    mf.mf_phase_timing(True)
    ms_per_step = timed(lambda: mf.mf_fastmm(algo, args.depth, args.cutoff, A, B, C), args.steps, 0)
    mf.mf_phase_timing(False)
    phase_ms, calls = mf.mf_phase_timing_read()
    phase_avg = [x / max(1, calls) for x in phase_ms]

    flops = 2.0 * n ** 3
    value = flops / (ms_per_step * 1e-3) / 1e9
    # algorithmic work of the dominant kernel: R^d leaf products of size n/2^d
    R = algo.info()["R"]
    p = algo.info()["n0"]
    d = args.depth
    m_true = n / p ** d
    gemm_flops = R ** d * 2.0 * m_true ** 3
    gemm_tflops = gemm_flops / (phase_avg[1] * 1e-3) / 1e12
    workload = f"fp64 n={n} {args.algo} depth {d}"
    roofline = {"bound": "mfma", "achieved": round(gemm_tflops, 2), "peak": FP64_MFMA_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(gemm_tflops / FP64_MFMA_PEAK_TFLOPS, 4),
                "traffic": traffic_for(workload), "kernel": "gemm_grouped<double>",
                "kernel_ms": round(phase_avg[1], 4)}

    # pre-addition phase against HBM: read A and B once, write the materialised blocks
    mat = mf.mf_workspace_bytes(algo, d, args.cutoff, n)  # includes group outputs when split
    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": workload, "n": n, "algo": args.algo, "depth": d, "cutoff": args.cutoff,
                   "storage": "fp64", "leaf": "fp64 MFMA", "inputs": "uniform[-1,1] seeds 10, 11"},
        "classical_ms": round(classical_ms, 4),
        "classical_gflops": round(flops / (classical_ms * 1e-3) / 1e9, 1),
        "speedup_vs_classical": round(classical_ms / ms_per_step, 4),
        "phases_ms": {"preadd": round(phase_avg[0], 4), "gemm": round(phase_avg[1], 4),
                      "postadd": round(phase_avg[2], 4)},
        "workspace_bytes": mat,
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        C_host = C.cpu().numpy()
        cb, err = cpu_baseline(args, A_host, B_host, C_host)
        out["cpu_baseline"] = cb
        out["rel_err"] = float(f"{err:.3e}")
    print(json.dumps(out), flush=True)


# ---------------------------------------------------------------------------
# Batched form: 512 uneven products in one persistent launch per dtype.
# ---------------------------------------------------------------------------

BATCH_COUNT, BATCH_SEED, BATCH_OPERAND_SEED = 512, 30, 31
FP32_MFMA_PEAK_TFLOPS = 157.3


def batch_operand_seeds(i):
    """Counter-generator seeds of instance i's A and B."""
    return 2 * (BATCH_OPERAND_SEED + i), 2 * (BATCH_OPERAND_SEED + i) + 1


def run_batched(args):
    import numpy as np
    import torch

    import mf_inputs as mi
    from paper_2312_12732_amd import mf

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    timed = timer(torch, stream)
    sizes = mi.batch_sizes(BATCH_COUNT, BATCH_SEED)
    wino = mf.mf_algo_builtin("winograd")
    R = 7
    flops = sum(2.0 * n ** 3 for n in sizes)
    per_dtype = {}
    for name, code, tdt, peak in (("f64", mf.MF_F64, torch.float64, FP64_MFMA_PEAK_TFLOPS),
                                  ("f32", mf.MF_F32, torch.float32, FP32_MFMA_PEAK_TFLOPS)):
        distinct = sorted(set(sizes))
        t0 = time.perf_counter()
        choices, tune_ms = mf.mf_autotune_batch(distinct, code, [wino], 3)
        tune_s = time.perf_counter() - t0
        pick = dict(zip(distinct, choices))
        As, Bs, Cs = [], [], []
        for i, n in enumerate(sizes):
            sa, sb = batch_operand_seeds(i)
            A = torch.empty(n, n, dtype=tdt, device=dev)
            B = torch.empty(n, n, dtype=tdt, device=dev)
            mf.mf_fill_uniform(A, sa)
            mf.mf_fill_uniform(B, sb)
            As.append(A)
            Bs.append(B)
            Cs.append(torch.empty_like(A))
        algos = [pick[n][0] for n in sizes]
        depths = [pick[n][1] for n in sizes]
        tuned = mf.mf_batch_create(sizes, algos, depths, [0] * len(sizes), code)
        plain = mf.mf_batch_create(sizes, [None] * len(sizes), [0] * len(sizes), [0] * len(sizes), code)
        ms_tuned = timed(lambda: mf.mf_batch_run(tuned, As, Bs, Cs), args.steps, args.warmup)
        assert not tuned.aborted(), "tuned batch aborted"
        # sampled parity against the oracle (smallest, median and largest instance)
        order = np.argsort(sizes, kind="stable")
        errs = []
        for i in (int(order[0]), int(order[len(order) // 2]), int(order[-1])):
            errs.append(batch_instance_error(sizes[i], i, Cs[i], np.float64 if name == "f64" else np.float32))
        ms_plain = timed(lambda: mf.mf_batch_run(plain, As, Bs, Cs), args.steps, args.warmup)
        assert not plain.aborted(), "classical batch aborted"

        def standalone():
            for A, B, C in zip(As, Bs, Cs):
                mf.mf_classical_mm(A, B, C)
        ms_loop = timed(standalone, max(2, args.steps // 2), 1)
        # algorithmic leaf work of the tuned batch: R^d products of size n / 2^d each
        leaf_flops = sum((R / 8.0) ** d * 2.0 * n ** 3 for n, d in zip(sizes, depths))
        achieved = leaf_flops / (ms_tuned * 1e-3) / 1e12
        hist = {}
        for n in sizes:
            key = "classical" if pick[n][1] == 0 else f"winograd d{pick[n][1]}"
            hist[key] = hist.get(key, 0) + 1
        per_dtype[name] = {
            "ms_per_step": round(ms_tuned, 4),
            "gflops": round(flops / (ms_tuned * 1e-3) / 1e9, 1),
            "classical_batch_ms": round(ms_plain, 4),
            "classical_batch_gflops": round(flops / (ms_plain * 1e-3) / 1e9, 1),
            "standalone_classical_ms": round(ms_loop, 4),
            "standalone_classical_gflops": round(flops / (ms_loop * 1e-3) / 1e9, 1),
            "speedup_vs_classical_batch": round(ms_plain / ms_tuned, 4),
            "speedup_vs_standalone_loop": round(ms_loop / ms_tuned, 4),
            "plans": hist,
            "tuning_s": round(tune_s, 2),
            "tuning_crossovers": crossover_table(distinct, choices, tune_ms),
            "sampled_rel_err": [float(f"{e:.3e}") for e in errs],
            "roofline": {"bound": "mfma", "achieved": round(achieved, 2), "peak": peak, "unit": "TFLOP/s",
                         "frac": round(achieved / peak, 4), "traffic": None,
                         "kernel": f"batch_persistent<{'double' if name == 'f64' else 'float'}>",
                         "kernel_ms": round(ms_tuned, 4)},
        }
        del As, Bs, Cs
        torch.cuda.empty_cache()
    f64 = per_dtype["f64"]
    total_ms = f64["ms_per_step"] + per_dtype["f32"]["ms_per_step"]
    out = {
        "metric": "effective GFLOP/s (sum of 2n^3 / t) of 512 uneven products in one persistent launch",
        "value": f64["gflops"], "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": f64["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "batched: 512 products, n = 64 round(exp(U(ln 128, ln 2048)) / 64) (seed 30), "
                               "FP64 batch and FP32 batch, operands from the counter generator (seeds 2(31+i), "
                               "2(31+i)+1), autotuned (winograd, depth) per size",
                   "count": BATCH_COUNT, "total_flops": flops},
        "both_dtypes_ms": round(total_ms, 4),
        "per_dtype": per_dtype,
        "roofline": f64["roofline"],
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = batch_cpu_baseline(sizes, pick)
    print(json.dumps(out), flush=True)


def crossover_table(distinct, choices, tune_ms):
    """Compact view of the tuner's result: size -> [chosen depth, ms per product of each candidate]."""
    return {str(n): [c[1]] + [round(x, 5) for x in ms] for n, c, ms in zip(distinct, choices, tune_ms)}


def batch_instance_error(n, i, C_dev, npdt):
    """Relative Frobenius error of instance i on 32 sampled rows against the
    oracle's definition rows (inputs regenerated on the host)."""
    import numpy as np

    import mf_inputs as mi
    from oracle import matmul as om

    sa, sb = batch_operand_seeds(i)
    A = mi.counter_uniform(n * n, sa, npdt).astype(np.float64).reshape(n, n)
    B = mi.counter_uniform(n * n, sb, npdt).astype(np.float64).reshape(n, n)
    rows = np.sort(np.random.default_rng(i).choice(n, size=min(n, 32), replace=False))
    return om.rel_fro_error(C_dev.cpu().numpy().astype(np.float64)[rows], om.rows_reference(A, B, rows))


def batch_cpu_baseline(sizes, pick):
    """Oracle fast products of the FP64 batch, in instance order, for about 10 s."""
    import numpy as np

    import mf_inputs as mi
    from oracle import algebra as oa
    from oracle import matmul as om

    U, V, W, conv = mi.as_float_tables(mi.WINOGRAD)
    alg = oa.canonical(2, U, V, W, conv)
    done, work, elapsed = 0, 0.0, 0.0
    for i, n in enumerate(sizes):
        if elapsed >= 10.0:
            break
        sa, sb = batch_operand_seeds(i)
        A = mi.counter_uniform(n * n, sa, np.float64).reshape(n, n)
        B = mi.counter_uniform(n * n, sb, np.float64).reshape(n, n)
        t0 = time.perf_counter()
        om.fast_mm(A, B, alg, pick[n][1], 0)
        elapsed += time.perf_counter() - t0
        work += 2.0 * n ** 3
        done += 1
    return {"value": round(work / elapsed / 1e9, 2), "unit": "GFLOP/s", "cores": oracle_cores(), "kind": "oracle",
            "sample": f"first {done} of {len(sizes)} FP64 instances with the tuned plans, oracle fast_mm "
                      f"(numpy/OpenBLAS float64), {elapsed:.1f} s"}


# ---------------------------------------------------------------------------
# Serving form: Poisson arrivals of mixed-size requests.
# ---------------------------------------------------------------------------

SERVE_SEED, SERVE_ARRIVAL_SEED = 40, 41
SERVE_SLOTS = 8
SERVE_BUDGET = 96 << 30
# depth k + 1 for n >= threshold k (FP64 and FP32 requests)
SERVE_POLICY = dict(depth_min_n_f64=(2048, 4096, 0, 0), depth_min_n_f32=(2048, 4096, 0, 0))


def run_serving(args):
    import numpy as np

    from paper_2312_12732_amd import mf
    import mf_inputs as mi

    reqs = mi.serving_requests(args.requests, SERVE_SEED)
    ns = [n for n, _ in reqs]
    codes = [mf.MF_F32 if d == "f32" else mf.MF_F64 for _, d in reqs]
    seeds = list(range(1, len(reqs) + 1))
    wino = mf.mf_algo_builtin("winograd")
    count = len(reqs)
    flops = sum(2.0 * n ** 3 for n in ns)

    def replay(slots, algo, policy, arrivals):
        srv = mf.Server(slots, SERVE_BUDGET, algo, **policy)
        srv.replay(arrivals, ns, codes, seeds)
        srv.drain()
        st = srv.stats()
        srv.close()
        return st

    zeros = np.zeros(count)
    replay(SERVE_SLOTS, wino, SERVE_POLICY, zeros)  # warm-up: plans, pool, code objects
    replay(SERVE_SLOTS, None, {}, zeros)
    ser = replay(1, wino, SERVE_POLICY, zeros)
    t_serial = ser["t_done"].max() - ser["t_admit"].min()
    mu = count / t_serial
    plain = replay(1, None, {}, zeros)
    t_plain = plain["t_done"].max() - plain["t_admit"].min()

    def summary(st, arrivals_start):
        lat = (st["t_done"] - st["t_arrive"]) * 1e3
        span = st["t_done"].max() - arrivals_start
        return {"p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3),
                "throughput_rps": round(count / span, 2), "gflops": round(flops / span / 1e9, 1)}

    rates = {}
    for k, f in enumerate((0.5, 0.9, 1.5)):
        arrivals = mi.poisson_arrivals(count, f * mu, SERVE_ARRIVAL_SEED + k)
        fast = replay(SERVE_SLOTS, wino, SERVE_POLICY, arrivals)
        base = replay(1, None, {}, arrivals)
        rates[f"{f}mu"] = {"lambda_rps": round(f * mu, 2),
                           "continuous_fast": summary(fast, fast["t_arrive"].min()),
                           "serial_classical": summary(base, base["t_arrive"].min())}
    top = rates["1.5mu"]["continuous_fast"]
    out = {
        "metric": "requests/s and p50/p99 latency of the serving loop under Poisson load",
        "value": top["throughput_rps"], "unit": "requests/s", "n_gpus": 1, "steps": count, "warmup": 2 * count,
        "ms_per_step": round(1e3 / top["throughput_rps"], 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64+f32", "data": "synthetic",
        "config": {"workload": f"serving: {count} requests, n = round(exp(U(ln 256, ln 8192))), 70% FP32 / 30% FP64 "
                               f"(seed {SERVE_SEED}), Poisson arrivals at 0.5, 0.9, 1.5 x the serial service rate "
                               f"(seeds {SERVE_ARRIVAL_SEED}+k), {SERVE_SLOTS} slots, budget {SERVE_BUDGET >> 30} GiB",
                   "policy": SERVE_POLICY},
        "serial_fast_s": round(t_serial, 4), "serial_classical_s": round(t_plain, 4),
        "mu_serial_rps": round(mu, 2), "rates": rates,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = serving_cpu_baseline(reqs, seeds)
    print(json.dumps(out), flush=True)


def serving_cpu_baseline(reqs, seeds):
    """Oracle products of the requests in arrival order, for about 10 s."""
    import numpy as np

    import mf_inputs as mi
    from oracle import algebra as oa
    from oracle import matmul as om

    U, V, W, conv = mi.as_float_tables(mi.WINOGRAD)
    alg = oa.canonical(2, U, V, W, conv)
    thr = SERVE_POLICY["depth_min_n_f64"]
    done, elapsed = 0, 0.0
    for (n, dt), seed in zip(reqs, seeds):
        if elapsed >= 10.0:
            break
        npdt = np.float64 if dt == "f64" else np.float32
        A = mi.counter_uniform(n * n, 2 * seed, npdt).astype(np.float64).reshape(n, n)
        B = mi.counter_uniform(n * n, 2 * seed + 1, npdt).astype(np.float64).reshape(n, n)
        depth = sum(1 for t in thr if t and n >= t)
        t0 = time.perf_counter()
        om.fast_mm(A, B, alg, depth, 0)
        elapsed += time.perf_counter() - t0
        done += 1
    return {"value": round(done / elapsed, 3), "unit": "requests/s", "cores": oracle_cores(), "kind": "oracle",
            "sample": f"first {done} of {len(reqs)} requests, served one after another by the oracle fast_mm "
                      f"(float64) with the same depth policy, {elapsed:.1f} s"}


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(the sharding design is described in DESIGN.md).", file=sys.stderr)
        sys.exit(2)
    if args.workload == "square":
        run_square(args)
    elif args.workload == "batched":
        run_batched(args)
    else:
        run_serving(args)


if __name__ == "__main__":
    main()
