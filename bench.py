"""Throughput of the SSM particle step on one MI355X.

One step = one time step (2.3)-(2.4) of the whole particle system: implicit
solve, O(N^2) interaction at mu^Y, diffusion, Brownian increments and the
explicit update.  Default workload: d=1, N=2^16 particles, T=1, h=2^-10 (1024
steps), Gaussian-interaction coefficients, pairwise sums in FP32 with
compensated accumulation; X_0 and the Brownian paths are seeded Philox draws.

Prints one JSON line.  value = particle-steps/s over the timed steps.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3   # MI355X vector FP32 (published)
PEAK_FP64_TFLOPS = 78.6


def flops_per_pair(d: int) -> int:
    """Algorithmic work of one interaction pair: d subtractions, d squares and
    d-1 adds, one scale, one exp, d multiplies and d accumulates."""
    return 5 * d + 1


def kernel_sources_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in ("ssm_kernels.hpp", "ssm_device.hpp"):
        with open(os.path.join(ROOT, "paper_2105_09688_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic(key: str):
    """HBM bytes per launch of the pair kernel from the committed rocprofv3
    FETCH_SIZE/WRITE_SIZE runs, if the kernel sources are unchanged since."""
    try:
        with open(os.path.join(ROOT, "profiles", "traffic.json")) as fh:
            rec = json.load(fh).get(key)
    except (OSError, ValueError):
        return None
    if not rec or rec.get("kernel_sources_sha256") != kernel_sources_sha256():
        return None
    return rec["hbm_bytes_per_launch"]


def cpu_baseline(w, budget_s: float):
    """The FP64 oracle on this host's cores, on a bounded sample of the same
    workload: whole time steps of the same system, as many as fit in the budget."""
    import numpy as np
    import oracle
    N, ens, h = w["systems"][0]
    X = oracle.init_state(w, ens, N)
    t0 = time.perf_counter()
    steps = 0
    while True:
        X, _ = oracle.step(w, ens, h, steps, X)
        steps += 1
        if time.perf_counter() - t0 >= budget_s or steps >= 8:
            break
    dt = time.perf_counter() - t0
    assert np.all(np.isfinite(X))
    return {"value": N * steps / dt, "unit": "particle-steps/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"{steps} full time steps of the same system (N={N}, d={w['d']}), FP64, from X_0"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1024)
    ap.add_argument("--warmup", type=int, default=16)
    ap.add_argument("--precision", default="fp32_kahan", choices=["fp64", "fp32", "fp32_kahan"])
    ap.add_argument("--N", type=int, default=2 ** 16)
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="after the run, one plain device copy of this many MiB (calibrates byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(the per-step all-gather of Y* across GPUs is a design note, not code).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2105_09688_amd import workloads as W
    from paper_2105_09688_amd.ssm import SSM

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    w = W.single_gpu_d1(N=args.N)
    N, _, h = w["systems"][0]
    d = w["d"]
    total_steps = int(round(w["T"] / h))
    if not (1 <= args.steps <= total_steps):
        raise SystemExit(f"--steps must be in 1..{total_steps} (T/h)")

    stream = torch.cuda.Stream()
    # warm-up (separate context: the timed one starts at t = 0)
    with SSM(w, precision=args.precision, stream=stream) as s:
        s.step(min(args.warmup, total_steps))
        s.sync()
    s = SSM(w, precision=args.precision, stream=stream)
    s.sync()
    s.profile(True)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    t0 = time.perf_counter()
    s.step(args.steps)
    ev1.record(stream)
    s.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    info = s.info()
    elapsed = gpu_ms / 1e3

    pair_avg_s = info["pair_ms"] / 1e3 / max(1, info["pair_launches"])
    pairs = float(N) * float(N)
    flop = pairs * flops_per_pair(d)
    achieved = flop / pair_avg_s / 1e12
    peak = PEAK_FP64_TFLOPS if args.precision == "fp64" else PEAK_FP32_TFLOPS

    out = {
        "metric": "particle-steps/s (SSM time steps of the N-particle system, exact O(N^2) interaction)",
        "value": N * args.steps / elapsed,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": gpu_ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "fp32_kahan": "f32 (compensated sums)"}[args.precision],
        "data": "synthetic (seeded Philox X_0 ~ N(1, 0.5^2) and Brownian paths)",
        "config": {"workload": f"SSM d={d} N={N} T=1 h=2^-10 Gaussian interaction (l=1), cubic v, "
                               f"affine sigma; {args.precision}",
                   "d": d, "N": N, "h": h, "T": w["T"], "precision": args.precision},
        "wall_s": wall,
        "roofline": {
            "bound": "alu",
            "kernel": "k_pair (O(N^2) interaction sums)",
            "achieved": achieved,
            "peak": peak,
            "unit": "TFLOP/s",
            "frac": achieved / peak,
            "traffic": recorded_traffic(f"k_pair {args.precision} d={d} N={N} R={info['targets_per_lane']} "
                                        f"L={info['sources_per_item']}"),
            "flop_per_pair": flops_per_pair(d),
            "pairs_per_launch": pairs,
            "avg_launch_ms": pair_avg_s * 1e3,
            "launches": info["pair_launches"],
        },
        "update_kernel_avg_ms": info["update_ms"] / max(1, info["update_launches"]),
        "tiling": {"targets_per_lane": info["targets_per_lane"], "sources_per_item": info["sources_per_item"],
                   "wavefront_items": info["n_pair_items"]},
    }
    if not args.no_check and args.precision != "fp64":
        # pathwise agreement of the timed run with the FP64 path after the same steps
        with SSM(w, precision="fp64", stream=stream) as ref:
            ref.step(args.steps)
            ref.sync()
            a, b = s.state(0), ref.state(0)
        out["check"] = {"max_pathwise_err_vs_fp64": float(np.max(np.abs(a - b) / np.maximum(1.0, np.abs(b)))),
                        "steps": args.steps}
    s.close()
    if args.calib_copy_mib > 0:
        n = args.calib_copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["calib_copy_bytes"] = {"read": 4 * n, "write": 4 * n}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
