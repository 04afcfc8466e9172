"""Autotuner of the pairwise kernel's tiling (targets per lane, sources per
work item, ordered or symmetric pair scheme).

Candidates are timed with the library's own per-kernel HIP events on a fresh
context of the workload; the fastest is cached in a JSON file keyed by the
workload shape, precision and GPU architecture ($SSM_TUNE_CACHE, default
~/.cache/ssm_tune.json).  Results do not depend on the tiling beyond
floating-point summation order (tested), so any cached choice is safe.
"""
from __future__ import annotations

import json
import os

from .ssm import SSM


def _cache_path() -> str:
    return os.environ.get("SSM_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "ssm_tune.json"))


def _key(workload: dict, precision: str) -> str:
    import torch
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    Ns = sorted(int(s[0]) for s in workload["systems"])
    hs = sorted({float(s[2]) for s in workload["systems"]})
    return json.dumps({"d": workload["d"], "N": Ns[:8] + ([len(Ns), sum(Ns)] if len(Ns) > 8 else []),
                       "levels": len(hs), "precision": precision, "arch": arch}, sort_keys=True)


def candidates(d: int, precision: str):
    out = []
    for scheme in ("symmetric", "ordered"):
        # symmetric: a target group (4 x 64 R particles) times d must fit the LDS row
        # (2048 floats, 3072 for d = 3, where R = 4 fits but measured slower than R = 2;
        # 1024 doubles, 1536 for d = 3)
        if scheme == "ordered":
            Rs = (2, 4) if d == 1 else (1, 2)
        elif precision == "fp64":
            Rs = {1: (1, 2, 4), 2: (1, 2), 3: (1, 2)}.get(d, (1,))
        else:
            Rs = {1: (2, 4, 8), 2: (1, 2, 4)}.get(d, (1, 2))
        for R in Rs:
            for Lmul in (0.5, 1.0, 2.0):
                out.append({"pair_scheme": scheme, "targets_per_lane": R, "L_factor": Lmul})
    return out


def measure(workload: dict, precision: str, cand: dict, stream=None, steps: int = 24) -> float:
    """Average time (ms) per tick of the pair and update kernels of `cand`
    over `steps` ticks after one warm tick (the tiling sets both: the update
    kernel combines the pair kernel's partial sums)."""
    kw = dict(precision=precision, stream=stream, targets_per_lane=cand["targets_per_lane"],
              pair_scheme=cand["pair_scheme"])
    with SSM(workload, **kw) as s:
        L0 = s.info()["sources_per_item"]
    unit = 16 if cand["pair_scheme"] == "symmetric" else 64
    L = max(unit * 4, int(L0 * cand["L_factor"]) // unit * unit)
    cand["sources_per_item"] = L
    with SSM(workload, sources_per_item=L, **kw) as s:
        ticks = s.info()["ticks_total"]
        n = min(steps, ticks - 1)
        s.step(1)
        s.sync()
        s.profile(True)
        s.step(n)
        s.sync()
        i = s.info()
    return (i["pair_ms"] + i["update_ms"]) / max(1, i["pair_launches"])


def autotune(workload: dict, precision: str = "fp32_kahan", stream=None, steps: int = 24,
             use_cache: bool = True, verbose: bool = False) -> dict:
    """Best tiling for `workload`: {"targets_per_lane", "sources_per_item", "pair_scheme"}."""
    key = _key(workload, precision)
    path = _cache_path()
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            with open(path) as fh:
                cache = json.load(fh)
        except (OSError, ValueError):
            cache = {}
        if key in cache:
            return cache[key]
    best, best_ms = None, float("inf")
    for cand in candidates(workload["d"], precision):
        ms = measure(workload, precision, cand, stream=stream, steps=steps)
        if verbose:
            print(f"[tune] {cand} -> {ms:.4f} ms", flush=True)
        if ms < best_ms:
            best_ms, best = ms, cand
    choice = {"targets_per_lane": best["targets_per_lane"], "sources_per_item": best["sources_per_item"],
              "pair_scheme": best["pair_scheme"], "tick_ms": best_ms}
    cache[key] = choice
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        with open(path, "w") as fh:
            json.dump(cache, fh, indent=1)
    except OSError:
        pass
    return choice
