"""Writes fixed_rmse.json: the FP64 oracle's strong errors (epsilon_2 of
Section 3, terminal time, over all particles) of two reduced workloads, each
against a proxy solution on the same Brownian paths.  They are the "fixed
rMSE" that the surrogate and batched runs are held to (within 5 %) by the
benchmark's reduced-size legs and by the GPU tests.  Only the oracle is
called; the inputs are the seeded workloads.

  python tests/golden/make_fixed_rmse.py      (about 15 minutes on 8 cores)
"""
import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2105_09688_amd import workloads as W  # noqa: E402


def surrogate_reduced(N=8192):
    """The surrogate case's coefficients (d = 2, h = 2^-9, T = 1) at N = 8192
    (the smallest size at which most of a network's checks meet the 1e-3
    tolerance: the finite-N part of the pair term, which no function of the
    moments can follow, shrinks with N), against a 2^-13 proxy."""
    w = W.surrogate_d2(N=N, h=2.0 ** -9, h_fine=2.0 ** -13)
    o = oracle.run(w)[0]
    o_ref = oracle.run(W.with_h(w, 2.0 ** -13))[0]
    return {"workload": f"surrogate case coefficients, d=2, N={N}, ensemble 0, h=2^-9, T=1, seed 0",
            "proxy_h": 2.0 ** -13, "N": N, "h": 2.0 ** -9, "T": 1.0,
            "rmse": oracle.strong_error(o, o_ref), "weak": oracle.weak_error(o, o_ref)}


def batched_reduced():
    """The batched case's coefficients and step sizes (h = 2^-4 .. 2^-8 on a
    2^-12 grid, T = 1) for 8 ensembles of N log-uniform in [2^8, 2^11],
    per step size against the 2^-12 proxy of each ensemble."""
    levels = (4, 5, 6, 7, 8)
    sizes = W.batched_sizes(n_ens=8, lo_log2=8, hi_log2=11)
    w = W.batched(n_ens=len(sizes), levels=levels, h_fine=2.0 ** -12, sizes=sizes)
    ref_w = W.with_systems(w, [(N, e, 2.0 ** -12) for e, N in enumerate(sizes)])
    o = oracle.run(w)
    o_ref = oracle.run(ref_w)
    per = {}
    for li, l in enumerate(levels):
        sq, cnt = 0.0, 0
        for e, N in enumerate(sizes):
            X = o[e * len(levels) + li]
            sq += float(((X - o_ref[e]) ** 2).sum())
            cnt += N
        per[f"2^-{l}"] = math.sqrt(sq / cnt)
    return {"workload": "batched case coefficients, d=1, 8 ensembles, N = batched_sizes(8, 8, 11), "
                        "h=2^-4..2^-8, h_fine=2^-12, T=1, seed 0",
            "sizes": sizes, "levels": list(levels), "proxy_h": 2.0 ** -12, "rmse": per}


def main():
    out = {"generator": "tests/golden/make_fixed_rmse.py (FP64 oracle only)"}
    for name, fn in (("surrogate_reduced", surrogate_reduced), ("batched_reduced", batched_reduced)):
        t0 = time.perf_counter()
        out[name] = fn()
        out[name]["oracle_seconds"] = round(time.perf_counter() - t0, 1)
        print(name, out[name], flush=True)
    with open(os.path.join(HERE, "fixed_rmse.json"), "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")


if __name__ == "__main__":
    main()
