"""Benchmark: condensed-IPM solves per second on one MI355X.

One step = one complete solve of the 1-D heat MPC problem with ns = 1000 states, nu = 10
inputs, horizon N = 50 (K is 500 x 500, Gamma has 50,000 rows): set the initial state
(x0 already resident in HBM) and run the interior-point method to tol 1e-8.  Each step uses
a different seeded x0.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--precision fp64] [--no-cpu-baseline]

The dominant kernel is the stream-K SYRK that forms K; its duration is measured with HIP
events on the library's stream over the timed solves and priced against the FP64 MFMA peak
with the structural FLOP count (only the nonzero blocks of Gamma).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "condensed-IPM solves/s & ms/iter (SYRK+POTRF) at tol 1e-8; mixed vs FP64"
PEAK = {"fp64": 78.6, "fp32": 157.3}          # MI355X dense MFMA, TFLOP/s
PRECISIONS = {"fp64": 0, "fp32": 1}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "syrk_f64_heat1d_ns1000_traffic.json")


def kernel_source_hash() -> str:
    path = os.path.join(ROOT, "paper_2209_13049_amd", "csrc", "k_syrk.hip")
    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]


def measured_traffic():
    """HBM bytes per SYRK launch from rocprofv3 counters, if they were taken on the current
    kernel source (else None)."""
    try:
        rec = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(p, solves: int = 1):
    """The CPU oracle, timed on the host on a bounded sample of the same workload."""
    import numpy as np
    import oracle
    from paper_2209_13049_amd import workloads as W
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()
                       if i.get("internal_api") in ("openblas", "mkl", "blis")] or [1])
    except Exception:
        threads = len(os.sched_getaffinity(0))
    total, iters = 0.0, 0
    for k in range(solves):
        pk = W.heat1d_config("1d", instance=k)
        red = oracle.reduce_problem(pk)
        t0 = time.perf_counter()
        r = oracle.solve(pk, red=red)
        total += time.perf_counter() - t0
        iters += r.iters
    return {"value": solves / total, "unit": "solves/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{solves} full oracle solve(s) of the same workload (instances 0..{solves - 1}, "
                      f"{iters} iterations; state elimination built beforehand, not timed)",
            "s_per_iter": total / max(1, iters)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--precision", default="fp64", choices=sorted(PRECISIONS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-solves", type=int, default=1)
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the timed run at the other precision")
    ap.add_argument("--calib-copy", action="store_true",
                    help="first run a plain elementwise copy of 256 MiB (reference for the "
                         "hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; the multi-GPU "
                                   "sharding is a design note only (no collectives are built)",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2209_13049_amd import condmpc
    from paper_2209_13049_amd import workloads as W

    torch.cuda.set_device(0)
    if args.calib_copy:
        a = torch.ones(32 * 2**20, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        del a, b
    cfg = W.CONFIG_1D
    base = W.heat1d_config("1d", instance=0)
    prob = condmpc.Problem(base)
    info = prob.info()
    total = args.warmup + args.steps
    x0s = [torch.from_numpy(W.heat1d_config("1d", instance=k).x0).to("cuda:0")
           for k in range(total)]

    def run(precision):
        """Warm up, then time `steps` solves (each: set x0, solve) at one precision."""
        opts = condmpc.default_options(precision=PRECISIONS[precision], profile=1)
        res = condmpc.Result()
        objs = []

        def step(k):
            prob.set_x0(x0s[k])
            rc = prob.solve_raw(opts, res)
            if rc != condmpc.OK:
                raise RuntimeError(f"solve {k} returned {rc}: {condmpc.load().cmpc_last_error()}")
            return res.iters, res.ms_syrk, res.ms_form, res.ms_potrf, res.obj

        for k in range(args.warmup):
            step(k)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        acc = np.zeros(4)
        for k in range(args.warmup, total):
            it, a, b, c, f = step(k)
            acc += (it, a, b, c)
            objs.append(f)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        iters = max(1.0, acc[0])
        syrk_avg_s = acc[1] / 1e3 / iters
        achieved = info["syrk_flops"] / syrk_avg_s / 1e12
        return {"solves_per_s": args.steps / elapsed, "ms_per_step": elapsed * 1e3 / args.steps,
                "iters_per_solve": acc[0] / args.steps, "ms_per_iter": elapsed * 1e3 / iters,
                "ms_per_iter_syrk_potrf": (acc[2] + acc[3]) / iters,
                "ms_per_iter_syrk_kernel": acc[1] / iters, "ms_per_iter_potrf": acc[3] / iters,
                "syrk_achieved_tflops": achieved, "syrk_avg_launch_us": syrk_avg_s * 1e6,
                "objs": objs}

    main_run = run(args.precision)
    other = "fp32" if args.precision == "fp64" else "fp64"
    other_run = run(other) if not args.no_compare else None
    peak = PEAK[args.precision]
    achieved = main_run["syrk_achieved_tflops"]
    out = {
        "metric": METRIC,
        "value": main_run["solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_run["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32-syrk/f64",
        "data": "synthetic",
        "config": {"workload": f"heat1d_ns{cfg['ns']}_nu{cfg['nu']}_N{cfg['N']}",
                   "ns": cfg["ns"], "nu": cfg["nu"], "N": cfg["N"], "n": info["n"],
                   "state_rows": info["mx"], "tol": 1e-8, "precision": args.precision,
                   "x0": "U(-0.4, 0.4) per state, seed [1, step]"},
        "iters_per_solve": main_run["iters_per_solve"],
        "ms_per_iter": main_run["ms_per_iter"],
        "ms_per_iter_syrk_potrf": main_run["ms_per_iter_syrk_potrf"],
        "ms_per_iter_syrk_kernel": main_run["ms_per_iter_syrk_kernel"],
        "ms_per_iter_potrf": main_run["ms_per_iter_potrf"],
        "roofline": {"bound": "mfma", "kernel": "syrk_streamk_kernel<double>" if
                     args.precision == "fp64" else "syrk_streamk_kernel<float>",
                     "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": measured_traffic() if
                     args.precision == "fp64" else None,
                     "flops_per_launch": info["syrk_flops"],
                     "avg_launch_us": main_run["syrk_avg_launch_us"]},
    }
    if other_run is not None:
        rel = [abs(a - b) / max(1.0, abs(b)) for a, b in zip(other_run["objs"], main_run["objs"])]
        out["compare"] = {
            "precision": other,
            "solves_per_s": other_run["solves_per_s"],
            "speedup_vs_" + args.precision: other_run["solves_per_s"] / main_run["solves_per_s"],
            "iters_per_solve": other_run["iters_per_solve"],
            "ms_per_iter": other_run["ms_per_iter"],
            "ms_per_iter_syrk_potrf": other_run["ms_per_iter_syrk_potrf"],
            "syrk_kernel_us": other_run["syrk_avg_launch_us"],
            "syrk_achieved_tflops_structural": other_run["syrk_achieved_tflops"],
            "syrk_peak_tflops": PEAK[other],
            "max_obj_rel_diff": max(rel) if rel else None,
        }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(base, args.cpu_solves)
    prob.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
