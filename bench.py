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


PROFILE_EVERY = 8  # ticks between timed pair launches in the headline run


def flops_per_pair(d: int) -> int:
    """Algorithmic work of one interaction pair: d subtractions, d squares and
    d-1 adds, one scale, one exp, d multiplies and d accumulates."""
    return 5 * d + 1


ISSUE_LANE_OPS = 256 * 4 * 16 * 2.4e9  # non-packed VALU issue: CUs x SIMDs x lanes x clock


def issue_ceiling_tflops(d: int, scheme: str) -> float:
    """FP32 pair kernel's issue-bound ceiling in algorithmic TFLOP/s: without
    packed FP32 each lane issues one VALU op per slot; an unordered pair costs
    d subtractions, d multiply-adds for |z|^2, the exponential (2 slots, half
    rate) and 2d accumulations (symmetric: 2d + 1 slots per ordered pair), an
    ordered pair d + d + 2 + d (3d + 2 slots)."""
    slots = 2 * d + 1 if scheme == "symmetric" else 3 * d + 2
    return ISSUE_LANE_OPS / slots * flops_per_pair(d) / 1e12


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


def oracle_time_runs(ws, particle_steps_total):
    """CPU baseline of a study: the FP64 oracle timed on whole runs of the same
    workloads on this host's cores (results unused)."""
    import oracle
    t0 = time.perf_counter()
    for w in ws:
        oracle.run(w)
    dt = time.perf_counter() - t0
    return {"seconds": dt, "value": particle_steps_total / dt, "unit": "particle-steps/s",
            "cores": oracle.num_threads(), "kind": "oracle"}


def cpu_baseline(w, budget_s: float):
    """The FP64 oracle on this host's cores, on a bounded sample of the same
    workload: whole time steps of the same system from X_0, until the budget
    (default 12 s) is spent (at most 64 steps)."""
    import numpy as np
    import oracle
    N, ens, h = w["systems"][0]
    X = oracle.init_state(w, ens, N)
    t0 = time.perf_counter()
    steps = 0
    while True:
        X, _ = oracle.step(w, ens, h, steps, X)
        steps += 1
        if time.perf_counter() - t0 >= budget_s or steps >= 64:
            break
    dt = time.perf_counter() - t0
    assert np.all(np.isfinite(X))
    return {"value": N * steps / dt, "unit": "particle-steps/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"{steps} full time steps of the same system (N={N}, d={w['d']}), FP64, from X_0"}


def timed_run(SSM, w, precision, stream, steps=None, profile=True, setup=None, **kw):
    """Fresh context, then `steps` ticks (default: to T) between HIP events on its stream."""
    import torch
    s = SSM(w, precision=precision, stream=stream, **kw)
    if setup is not None:
        setup(s)
    s.sync()
    if profile:
        s.profile(True)
    info0 = s.info()
    n = info0["ticks_total"] if steps is None else steps
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    s.step(n)
    e1.record(stream)
    s.sync()
    torch.cuda.synchronize()
    return s, e0.elapsed_time(e1) / 1e3, n


def particle_steps(w, ticks):
    """sum over systems of N_s x (steps system s takes in `ticks` ticks)."""
    h_min = min(sy[2] for sy in w["systems"])
    tot = 0
    for N, _e, h in w["systems"]:
        stride = int(round(h / h_min))
        tot += N * ((ticks + stride - 1) // stride)
    return tot


def study_precision(args, stream):
    """d=3 precision study: FP64, FP32 and FP32-compensated runs of the same
    paths (the compensated mode also with every pair term compensated, on
    ordered pairs); errors of the FP32 modes against the FP64 path (mean,
    variance, rMSE)."""
    import numpy as np
    from paper_2105_09688_amd import workloads as W
    from paper_2105_09688_amd.ssm import SSM
    w = W.precision_d3(N=args.N or 2 ** 18)
    N = w["systems"][0][0]
    res = {}
    states = {}
    runs = (("fp64", "fp64", {}), ("fp32_kahan", "fp32_kahan", {}), ("fp32", "fp32", {}),
            ("fp32_kahan_per_pair", "fp32_kahan", {"kahan_span": 1}))
    for key, prec, kw in runs:
        s, dt, n = timed_run(SSM, w, prec, stream, **kw)
        info = s.info()
        states[key] = (s.state(0), s.moments(0))
        pair_avg = info["pair_ms"] / 1e3 / max(1, info["pair_launches"])
        res[key] = {"seconds": dt, "steps": n, "particle_steps_per_s": N * n / dt,
                    "pair_kernel_avg_ms": pair_avg * 1e3,
                    "pair_tflops": float(N) * N * flops_per_pair(3) / pair_avg / 1e12,
                    "pair_scheme": info["pair_scheme"]}
        s.close()
        print(f"[precision] {key}: {dt:.2f} s", file=sys.stderr, flush=True)
    X64, (m64, v64) = states["fp64"]
    for prec in ("fp32_kahan", "fp32", "fp32_kahan_per_pair"):
        X, (m, v) = states[prec]
        D = X - X64
        res[prec]["err_vs_fp64"] = {
            "mean_abs": [float(x) for x in np.abs(m - m64)],
            "var_abs": [float(x) for x in np.abs(v - v64)],
            "pathwise_rms": float(np.sqrt(np.sum(D * D) / N)),
            "pathwise_max_rel": float(np.max(np.abs(D) / np.maximum(1.0, np.abs(X64)))),
        }
    res["fp64"]["mean"] = [float(x) for x in m64]
    res["fp64"]["var"] = [float(x) for x in v64]
    return {"study": "precision", "workload": f"d=3 N={N} T=1 h=2^-10 l=0.5", "results": res}


def study_small(args, stream):
    """Small parity case (10 ensembles x N=1000, d=1, 256 steps, FP64; also
    FP32-compensated): whole-run time of the persistent launch (the library
    default at this size), of the multi-launch path with eager launches, and
    of the multi-launch path with per-tick graph replays; the first tick is
    not timed (it captures the graph)."""
    import numpy as np
    from paper_2105_09688_amd import workloads as W
    from paper_2105_09688_amd.ssm import SSM
    w = W.small_parity()
    out = {"study": "small", "workload": "10 ensembles x N=1000, d=1, h=2^-8, 256 steps"}
    modes = (("persistent", dict(persistent=1)), ("eager", dict(persistent=-1)),
             ("graphs", dict(persistent=-1, graphs=True)))
    for prec in ("fp64", "fp32_kahan"):
        finals = {}
        for name, kw in modes:
            s, dt, n = timed_run(SSM, w, prec, stream, steps=255, profile=False, setup=lambda c: c.step(1), **kw)
            finals[name] = s.states()
            s.close()
            out[f"{prec} {name}"] = {"seconds": dt, "particle_steps_per_s": 10 * 1000 * n / dt,
                                     "us_per_step": dt / n * 1e6}
        # the two paths differ by summation order only
        out[f"{prec} persistent vs eager, max pathwise difference"] = max(
            float(np.max(np.abs(a - b) / np.maximum(1.0, np.abs(b))))
            for a, b in zip(finals["persistent"], finals["eager"]))
    return out


def study_surrogate_tick(args, stream):
    """Cost of one surrogate tick at the surrogate case's size (d=2, N=2^20,
    FP32-compensated): one exact check tick, then 15 ticks on the network
    (residual mode, every check accepted), timed with the library's events.
    The weights are fresh (mlp_init): their accuracy does not change the work."""
    from paper_2105_09688_amd import workloads as W
    from paper_2105_09688_amd.ssm import SSM, mlp_init
    w = W.surrogate_d2(N=args.N or 2 ** 20)
    with SSM(w, precision="fp32_kahan", stream=stream) as s:
        s.surrogate_load(mlp_init(w["d"], seed=0))
        s.surrogate_enable(check_every=16, tol=1e9, mode="residual")
        s.step(1)
        s.sync()
        t0 = time.perf_counter()
        s.step(15)
        s.sync()
        dt = time.perf_counter() - t0
        info = s.info()
    return {"study": "surrogate_tick", "workload": f"d=2 N={w['systems'][0][0]} h=2^-9 fp32_kahan, residual mode",
            "surrogate_ticks": info["surr_ticks"], "ms_per_surrogate_tick": dt / 15 * 1e3}


def stability_beta(h, L_v, L_b, L_bt, L_s, L_st=0.0, L_vt=0.0):
    """beta of Theorem 2.9: sup_i E|X_n - Z_n|^2 <= (1 + beta h)^n sup_i E|X_0 - Z_0|^2,
    from the one-sided Lipschitz constant L_v of v, L_vt of its measure part,
    and the squared-Lipschitz constants of b and sigma in x (L_b, L_s) and in
    the measure (L_bt, L_st)."""
    den = 1.0 - h * (2.0 * L_v + 1.0)
    if not den > 0.0:
        raise ValueError("Theorem 2.9 needs 1 - h (2 L_v + 1) > 0")
    A = 2.0 * math.sqrt(L_b) + 2.0 * math.sqrt(L_bt) + L_s + L_st
    B = L_b + L_bt
    num = (2.0 * L_v + A + 1.0 + L_vt) + h * (L_vt * A + B) + h * h * B * L_vt
    return num / den


def gl_stability_beta(gamma, h):
    """beta of the Section 3.4.2 example: L_v = -5/2 - gamma, L_bt = L_s = 1,
    L_b = gamma^2, L_vt = L_st = 0."""
    return stability_beta(h, L_v=-2.5 - gamma, L_b=gamma * gamma, L_bt=1.0, L_s=1.0)


def _rmse(X, X_ref):
    """Strong error of Section 3 over the particles of all listed systems."""
    import numpy as np
    num = sum(float(np.sum((a - b) ** 2)) for a, b in zip(X, X_ref))
    return math.sqrt(num / sum(a.shape[-1] for a in X))


def _weak(X, X_ref):
    """Weak error of Section 3: norm of the mean difference over all particles."""
    import numpy as np
    D = np.concatenate([a - b for a, b in zip(X, X_ref)], axis=1)
    return float(np.linalg.norm(D.mean(axis=1)))


def _slope(hs, errs):
    import numpy as np
    return float(np.polyfit(np.log2(hs), np.log2(errs), 1)[0])


def study_families(args, stream):
    """The paper's own coefficient families (Section 3): stochastic
    Ginzburg-Landau in both SSM splittings (Section 3.1), polynomial drift
    (Section 3.3) and Cucker-Smale (Section 3.4.3, T = 2; also the mean and
    spread of V at T), N = 1000 x 10 ensembles, h = 2^-4 .. 2^-10 in one context,
    against a 2^-14 proxy on the same paths: strong and weak errors and their
    rates, and the GPU time; the oracle's time for the same runs is the CPU
    baseline.  (Parity of these runs with the oracle: tests/test_gpu_families.py.)"""
    from paper_2105_09688_amd import workloads as W
    from paper_2105_09688_amd.ssm import SSM
    prec = args.precision
    levels = (4, 5, 6, 7, 8, 9, 10)
    n_ens, N, hf = 10, 1000, 2.0 ** -14
    fams = {"ginzburg_landau_v1": lambda **k: W.ginzburg_landau(1, **k),
            "ginzburg_landau_v2": lambda **k: W.ginzburg_landau(2, **k),
            "polynomial_drift": lambda **k: W.polynomial_drift(**k),
            "cucker_smale": lambda **k: W.cucker_smale(**k)}
    out = {"study": "families", "workload": f"N={N} x {n_ens} ensembles, h=2^-4..2^-10, proxy 2^-14, T=1, {prec}"}
    for name, mk in fams.items():
        w = mk(n_ens=n_ens, N=N, h_fine=hf, levels=levels)
        ref_w = mk(n_ens=n_ens, N=N, h=hf, h_fine=hf)
        s, dt, n = timed_run(SSM, w, prec, stream, profile=False)
        r, dt_ref, n_ref = timed_run(SSM, ref_w, prec, stream, profile=False)
        g, g_ref = s.states(), r.states()
        s.close()
        r.close()
        res = {"levels": {}}
        hs, st, wk = [], [], []
        for li, l in enumerate(levels):
            sel = [g[e * len(levels) + li] for e in range(n_ens)]
            sg, wg = _rmse(sel, g_ref), _weak(sel, g_ref)
            res["levels"][f"2^-{l}"] = {"rmse": sg, "weak": wg}
            hs.append(2.0 ** -l)
            st.append(sg)
            wk.append(wg)
        if name == "cucker_smale":
            import numpy as np
            V = np.concatenate([x[0] for x in g_ref])
            res["V_at_T"] = {"mean": float(V.mean()), "std": float(V.std())}
        res["strong_slope"] = _slope(hs, st)
        res["weak_slope"] = _slope(hs, wk)
        ps = particle_steps(w, n) + particle_steps(ref_w, n_ref)
        res["gpu_seconds"] = dt + dt_ref
        res["gpu_particle_steps_per_s"] = ps / (dt + dt_ref)
        res["cpu_baseline"] = oracle_time_runs([w, ref_w], ps)
        out[name] = res
        print(f"[families] {name}: strong slope {res['strong_slope']:.3f}, weak slope {res['weak_slope']:.3f}, "
              f"gpu {dt + dt_ref:.2f} s, oracle {res['cpu_baseline']['seconds']:.2f} s", file=sys.stderr, flush=True)
    return out


def _series(SSM, w, prec, stream, times, wz=None):
    """E|X_t|^2 (and E|X_t - Z_t|^2 with a second context on the same paths)
    at the sampled times, averaged over particles and systems."""
    h = w["systems"][0][2]
    N = sum(sy[0] for sy in w["systems"])
    out = {"t": [], "m2": [], "msd": []}
    with SSM(w, precision=prec, stream=stream) as a:
        b = SSM(wz, precision=prec, stream=stream) if wz is not None else None
        try:
            tick = 0
            for t in times:
                n = int(round(t / h))
                if n > tick:
                    a.step(n - tick)
                    if b is not None:
                        b.step(n - tick)
                    tick = n
                m2 = 0.0
                for k, sy in enumerate(w["systems"]):
                    mean, var = a.moments(k)
                    m2 += sy[0] * float(sum(var) + sum(x * x for x in mean))
                out["t"].append(t)
                out["m2"].append(m2 / N)
                if b is not None:
                    out["msd"].append(sum(a.sqdiff(k, b, k) for k in range(len(w["systems"]))) / N)
        finally:
            if b is not None:
                b.close()
    if wz is None:
        del out["msd"]
    return out


def study_stability(args, stream):
    """Mean-square stability of the SSM (Theorem 2.9) on the example of
    Section 3.4.2, N = 1000 x 10 ensembles, FP64: (a) E|X_t|^2 for
    h = 1e-2, 1e-3, 1e-4 (gamma = 0, T = 3); (b) E|X_t - Z_t|^2 for X_0 = 1,
    Z_0 = 5, 10, 100 on the same paths (h = 1e-2) beside the bound
    (1 + beta h)^n |X_0 - Z_0|^2; (c) E|X_t|^2 for gamma = -12, 0, 12 at
    h = 0.1 to T = 15; (d) 1 + beta(gamma) h and E|X_T|^2 over gamma in
    [-12, 12] at h = 0.1, T = 3."""
    from paper_2105_09688_amd import workloads as W
    from paper_2105_09688_amd.ssm import SSM
    prec = "fp64" if args.precision == "fp32_kahan" else args.precision
    t0 = time.perf_counter()
    out = {"study": "stability", "workload": "Section 3.4.2 example, N=1000 x 10 ensembles, " + prec}
    ts3 = [0.25 * k for k in range(13)]
    out["a_h_sweep"] = {f"h={h:g}": _series(SSM, W.gl_stability(h=h), prec, stream, ts3)
                        for h in (1e-2, 1e-3, 1e-4)}
    h = 1e-2
    beta = gl_stability_beta(0.0, h)
    out["b_contraction"] = {"beta": beta, "one_plus_beta_h": 1 + beta * h}
    for z0 in (5.0, 10.0, 100.0):
        ser = _series(SSM, W.gl_stability(h=h), prec, stream, ts3, wz=W.gl_stability(h=h, x0=z0))
        ser["bound"] = [(1 + beta * h) ** int(round(t / h)) * (z0 - 1.0) ** 2 for t in ts3]
        out["b_contraction"][f"Z0={z0:g}"] = ser
    ts15 = [1.0 * k for k in range(16)]
    out["c_gamma_long"] = {f"gamma={g:g}": _series(SSM, W.gl_stability(gamma=g, h=0.1, T=15.0, allow_unstable_h=True),
                                                   prec, stream, ts15) for g in (-12.0, 0.0, 12.0)}
    d = {"gamma": [], "one_plus_beta_h": [], "m2_T": []}
    for g in range(-12, 13):
        ser = _series(SSM, W.gl_stability(gamma=float(g), h=0.1, allow_unstable_h=True), prec, stream, [3.0])
        d["gamma"].append(g)
        try:
            d["one_plus_beta_h"].append(1 + gl_stability_beta(float(g), 0.1) * 0.1)
        except ValueError:  # outside the step condition: no guarantee
            d["one_plus_beta_h"].append(None)
        d["m2_T"].append(ser["m2"][-1])
    out["d_gamma_sweep"] = d
    out["seconds"] = time.perf_counter() - t0
    return out


def study_batched(args, stream):
    """Batched case: 64 ensembles of uneven N x 5 step sizes in one context;
    throughput, and rMSE per step size against a 2^-12 proxy solution on the
    same Brownian paths, with the OLS slope."""
    import math
    from paper_2105_09688_amd import workloads as W
    from paper_2105_09688_amd.ssm import SSM
    levels = (4, 5, 6, 7, 8)
    w = W.batched(levels=levels)
    prec = args.precision
    # throughput without timing events, eager and with per-phase graph replays
    # (the first max_stride ticks, which capture the graphs, are not timed)
    rates = {}
    h_min = min(sy[2] for sy in w["systems"])
    ph = max(int(round(sy[2] / h_min)) for sy in w["systems"])
    n_total = int(round(w["T"] / h_min))
    for graphs in (False, True):
        g, dtg, ng = timed_run(SSM, w, prec, stream, steps=n_total - ph, profile=False, graphs=graphs,
                               setup=lambda c: c.step(ph))
        rates["graphs" if graphs else "eager"] = (particle_steps(w, n_total) - particle_steps(w, ph)) / dtg
        g.close()
    # profiled run: per-kernel times, and the final states for the errors
    s, dt, n = timed_run(SSM, w, prec, stream)
    info = s.info()
    ps = particle_steps(w, n)
    ref_w = W.with_systems(w, [(N, e, 2.0 ** -12) for (N, e) in {(sy[0], sy[1]) for sy in w["systems"]}])
    ref_w["systems"] = sorted(ref_w["systems"], key=lambda t: t[1])
    r, dt_ref, _ = timed_run(SSM, ref_w, prec, stream, profile=False)
    by_ens = {sy[1]: k for k, sy in enumerate(ref_w["systems"])}
    sq = {l: 0.0 for l in levels}
    cnt = {l: 0 for l in levels}
    for k, (N, e, h) in enumerate(w["systems"]):
        l = int(round(-math.log2(h)))
        sq[l] += s.sqdiff(k, r, by_ens[e])
        cnt[l] += N
    rmse = {l: math.sqrt(sq[l] / cnt[l]) for l in levels}
    xs = [math.log2(2.0 ** -l) for l in levels]
    ys = [math.log2(rmse[l]) for l in levels]
    xm, ym = sum(xs) / len(xs), sum(ys) / len(ys)
    slope = sum((x - xm) * (y - ym) for x, y in zip(xs, ys)) / sum((x - xm) ** 2 for x in xs)
    out = {"study": "batched", "workload": f"64 ensembles, N in [2^10, 2^16] (sum {sum(sy[0] for sy in w['systems']) // len(levels)}), "
                                            f"h = 2^-4..2^-8 on a 2^-12 grid, T=1, {prec}",
           "ticks": n, "particle_steps": ps,
           "particle_steps_per_s": rates["eager"], "particle_steps_per_s_graphs": rates["graphs"],
           "profiled_seconds": dt, "profiled_particle_steps_per_s": ps / dt,
           "pair_kernel_ms_total": info["pair_ms"], "update_kernel_ms_total": info["update_ms"],
           "rmse_vs_2^-12": {f"2^-{l}": rmse[l] for l in levels}, "slope": slope,
           "reference_seconds": dt_ref}
    s.close()
    r.close()
    return out


def training_snapshots(ticks: int) -> list:
    """Ticks at which the surrogate's training rows are drawn from an exact
    run: dense where the cloud changes fastest (X_0 ~ N(0, I) contracts under
    v = -|x|^2 x), every 2 ticks over the first 1/16 of the run, every 8 up to
    1/4, every 32 after (40 states for 512 ticks).  Measured on the surrogate
    case against 32 evenly spaced states at the same 2^22 rows: checks after
    16 and 32 steps dropped from 7.1e-3 / 1.8e-3 to 3.5e-3 / 0.9e-3 relative
    error (with the longer training), two fallback intervals instead of four."""
    e1, e2 = ticks // 16, ticks // 4
    s1, s2, s3 = max(1, ticks // 256), max(1, ticks // 64), max(1, ticks // 16)
    return list(range(0, e1, s1)) + list(range(e1, e2, s2)) + list(range(e2, ticks, s3))


def surrogate_training_rows(w, prec, stream, ensembles, N_train, rows_total):
    """(features, exact pair term) rows from exact runs of the given ensembles
    at N_train (same coefficients and step), drawn at training_snapshots."""
    import torch
    from paper_2105_09688_amd import workloads as W
    from paper_2105_09688_amd.ssm import SSM
    h = w["systems"][0][2]
    Us, Ts = [], []
    for e in ensembles:
        with SSM(W.with_systems(w, [(N_train, e, h)]), precision=prec, stream=stream) as s:
            snaps = training_snapshots(s.info()["ticks_total"])
            per = rows_total // (len(ensembles) * len(snaps))
            cur = 0
            for t in snaps:
                s.step(t - cur)
                cur = t
                U, T = s.surrogate_samples(per, seed=1000 * e + t)
                Us.append(U)
                Ts.append(T)
    return torch.cat(Us), torch.cat(Ts)


def study_surrogate(args, stream):
    """Learned surrogate (d=2, N=2^20, h=2^-9, T=1): training pairs from exact
    runs of other ensembles, Adam on the GPU, then the exact run and surrogate
    runs (exact check every 16 steps) of the same paths; beside the trained
    network, the same cadence and tolerances with an all-zero network in
    residual mode (the exact pair term frozen at the last check: the scheme
    without a network)."""
    import numpy as np
    import torch
    from paper_2105_09688_amd import workloads as W
    from paper_2105_09688_amd.ssm import SSM, mlp_init, mlp_train
    prec = args.precision
    w = W.surrogate_d2(N=args.N or 2 ** 20)
    N, _, h = w["systems"][0]
    d = w["d"]
    N_train, every = 2 ** 18, 16
    t0 = time.perf_counter()
    U, T = surrogate_training_rows(w, prec, stream, (1, 2), N_train, 2 ** 22)
    t_data = time.perf_counter() - t0
    print(f"[surrogate] {U.shape[0]} training pairs in {t_data:.1f} s", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    p = torch.tensor(mlp_init(d, seed=0), device="cuda")
    hist = []
    for steps, lr, seed in ((args.train_steps, 1e-3, 1), (args.train_steps // 2, 2e-4, 2), (args.train_steps // 4, 4e-5, 3)):
        hist.append(mlp_train(d, p, U, T, steps=steps, batch=4096, lr=lr, seed=seed))
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    hist = np.concatenate(hist)
    print(f"[surrogate] training {hist.size} steps in {t_train:.1f} s, loss {hist[:50].mean():.3e} -> "
          f"{hist[-200:].mean():.3e}", file=sys.stderr, flush=True)
    master = p.cpu().numpy()
    tsq = float(T.pow(2).sum(dim=1).mean())

    ex, dt_ex, n = timed_run(SSM, w, prec, stream)
    X_ex = ex.state(0)
    m_ex, v_ex = ex.moments(0)
    info_ex = ex.info()
    ex.close()
    print(f"[surrogate] exact run {dt_ex:.1f} s", file=sys.stderr, flush=True)
    runs = {}
    # the trained network, and (the scheme without a network) an all-zero
    # network in residual mode: the exact pair term frozen at the last check
    zeros = np.zeros_like(master)
    cases = (("gain", 1e-3, master, "", False), ("gain", 1e-2, master, "", False), ("gain", 1e9, master, "", False),
             ("residual", 1e-3, master, "", False), ("residual", 1e-3, master, "", True),
             ("residual", 1e9, master, "", False),
             ("residual", 1e-3, zeros, "frozen exact term, ", False),
             ("residual", 1e-3, zeros, "frozen exact term, ", True),
             ("residual", 1e9, zeros, "frozen exact term, ", False))
    for mode, tol, weights, tag, recheck in cases:
        def setup(s, tol=tol, mode=mode, weights=weights, recheck=recheck):
            s.surrogate_load(weights)
            s.surrogate_enable(check_every=every, tol=tol, mode=mode, recheck=recheck)
        su, dt_su, _ = timed_run(SSM, w, prec, stream, setup=setup)
        info = su.info()
        X = su.state(0)
        m, v = su.moments(0)
        su.close()
        D = X - X_ex
        runs[f"{tag}{mode} tol={tol:g}{' recheck' if recheck else ''}"] = {
            "seconds": dt_su, "particle_steps_per_s": N * n / dt_su, "speedup_vs_exact": dt_ex / dt_su,
            "checks": info["surr_checks"], "rechecks": info["surr_rechecks"], "surrogate_ticks": info["surr_ticks"],
            "fallback_ticks": info["surr_fallback_ticks"], "check_rel_err_last": info["surr_last_err"],
            "check_rel_err_max": info["surr_max_err"], "check_rel_err_last_without_gain": info["surr_last_raw_err"],
            "gain_last": info["surr_gain"],
            "pathwise_rms_vs_exact": float(np.sqrt(np.sum(D * D) / N)),
            "mean_diff": [float(x) for x in m - m_ex], "var_diff": [float(x) for x in v - v_ex],
        }
        print(f"[surrogate] {tag}{mode} tol {tol:g}{' recheck' if recheck else ''}: {dt_su:.2f} s, "
              f"{info['surr_ticks']} surrogate ticks, "
              f"last err {info['surr_last_err']:.3e}, max err {info['surr_max_err']:.3e}", file=sys.stderr, flush=True)
    # strong error at fixed h against a 2^-13 proxy solution on the same paths,
    # at N = min(N, 2^18), the size the network was trained at (the proxy run
    # takes 8192 exact steps)
    Nr = min(N, 2 ** 18)
    wr = W.with_systems(w, [(Nr, 0, h)])
    wr["h_fine"] = 2.0 ** -13
    ref = SSM(W.with_h(wr, 2.0 ** -13), precision=prec, stream=stream)
    ref.run()
    rm = {}
    variants = (("exact", None, None, None, False), ("gain tol=1e-2", "gain", 1e-2, master, False),
                ("gain always", "gain", 1e9, master, False), ("residual tol=1e-3", "residual", 1e-3, master, False),
                ("residual tol=1e-3 recheck", "residual", 1e-3, master, True),
                ("residual always", "residual", 1e9, master, False),
                ("frozen exact term tol=1e-3", "residual", 1e-3, zeros, False),
                ("frozen exact term always", "residual", 1e9, zeros, False))
    for label, mode, tol, weights, recheck in variants:
        with SSM(wr, precision=prec, stream=stream) as a:
            if tol is not None:
                a.surrogate_load(weights)
                a.surrogate_enable(check_every=every, tol=tol, mode=mode, recheck=recheck)
            a.run()
            rm[label] = math.sqrt(a.sqdiff(0, ref, 0) / Nr)
            if tol is not None:
                i = a.info()
                rm[label + " surrogate ticks"] = i["surr_ticks"]
    ref.close()
    for label, _m, tol, _w, _r in variants[1:]:
        rm[f"ratio {label} / exact"] = rm[label] / rm["exact"]
    pair_avg = info_ex["pair_ms"] / 1e3 / max(1, info_ex["pair_launches"])
    return {"study": "surrogate", f"rmse_vs_2^-13_at_N={Nr}": rm, "workload": f"d=2 N={N} T=1 h=2^-9, exact check every {every} steps, {prec}",
            "training": {"pairs": int(U.shape[0]), "from": f"exact runs of ensembles 1-2 at N={N_train}, "
                                                            "40 states each (training_snapshots)",
                         "data_seconds": t_data, "steps": int(hist.size), "batch": 4096,
                         "train_seconds": t_train, "loss_first": float(hist[:50].mean()),
                         "loss_last": float(hist[-200:].mean()), "target_mean_sq": tsq},
            "exact": {"seconds": dt_ex, "steps": n, "particle_steps_per_s": N * n / dt_ex,
                      "pair_kernel_avg_ms": pair_avg * 1e3,
                      "pair_tflops": float(N) * N * flops_per_pair(d) / pair_avg / 1e12},
            "surrogate": runs}


def golden_fixed_rmse(name: str) -> dict:
    """The oracle's strong errors of the reduced workloads, stored by
    tests/golden/make_fixed_rmse.py (which calls the oracle only)."""
    with open(os.path.join(ROOT, "tests", "golden", "fixed_rmse.json")) as fh:
        return json.load(fh)[name]


def settle_clocks(SSM, w, precision, stream, seconds: float) -> dict:
    """Untimed pair-kernel work until `seconds` of wall time have passed.  The
    kernel's duration falls by about 10 % over the first tens of milliseconds
    of sustained load (clock ramp: 401 -> 380 us over the first 20 launches
    at d = 1, N = 2^16, about 357 us from a few hundred on), so the timed
    steps start at steady clocks."""
    t0 = time.perf_counter()
    ticks = 0
    while time.perf_counter() - t0 < seconds:
        with SSM(w, precision=precision, stream=stream) as s:
            total = s.info()["ticks_total"]
            while time.perf_counter() - t0 < seconds and s.info()["tick"] < total:
                n = min(64, total - s.info()["tick"])
                s.step(n)
                s.sync()
                ticks += n
    return {"seconds": time.perf_counter() - t0, "ticks": ticks}


def _events(stream):
    import torch
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def _timed_steps(s, n, stream):
    """GPU time (s) of n ticks of context s, between HIP events on its stream."""
    import torch
    torch.cuda.synchronize()
    e0, e1 = _events(stream)
    e0.record(stream)
    s.step(n)
    e1.record(stream)
    s.sync()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3


def leg_surrogate(args, stream) -> dict:
    """The metric's surrogate leg on the surrogate case (d = 2, N = 2^20,
    h = 2^-9, T = 1, FP32-compensated): a network trained on exact runs of
    ensembles 1-2 at N = 2^18 (2^22 rows, Adam); the exact O(N^2) tick timed
    on 16 ticks; the whole surrogate run (residual mode, exact check every 16
    steps, fallback above 1e-3 relative drift error) timed from X_0 to T; the
    same run with rechecks (every fallback tick a check too); and the
    fixed-rMSE check at N = 8192 (same network, both rules) against the
    oracle's strong error stored in tests/golden/fixed_rmse.json, with the
    GPU's FP64 2^-13 run on the same paths as the proxy."""
    import numpy as np
    import torch
    from paper_2105_09688_amd import workloads as W
    from paper_2105_09688_amd.ssm import SSM, mlp_init, mlp_train
    prec = "fp32_kahan"
    w = W.surrogate_d2(N=2 ** 20)
    N, _, h = w["systems"][0]
    d = w["d"]
    every, tol = 16, 1e-3
    t0 = time.perf_counter()
    U, T = surrogate_training_rows(w, prec, stream, (1, 2), 2 ** 18, 2 ** 22)
    n_rows = int(U.shape[0])
    t_data = time.perf_counter() - t0
    t0 = time.perf_counter()
    p = torch.tensor(mlp_init(d, seed=0), device="cuda")
    hist = []
    for steps, lr, seed in ((args.train_steps, 1e-3, 1), (args.train_steps // 2, 2e-4, 2), (args.train_steps // 4, 4e-5, 3)):
        hist.append(mlp_train(d, p, U, T, steps=steps, batch=4096, lr=lr, seed=seed))
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    hist = np.concatenate(hist)
    master = p.cpu().numpy()
    del U, T
    print(f"[leg surrogate] {n_rows} rows in {t_data:.1f} s, {hist.size} Adam steps in {t_train:.1f} s", file=sys.stderr,
          flush=True)
    # exact ticks at full size
    with SSM(w, precision=prec, stream=stream) as ex:
        ex.step(1)
        ex.sync()
        n_ex = 16
        dt_ex = _timed_steps(ex, n_ex, stream)
    ms_exact = dt_ex / n_ex * 1e3
    # the whole surrogate run
    with SSM(w, precision=prec, stream=stream) as su:
        su.surrogate_load(master)
        su.surrogate_enable(check_every=every, tol=tol, mode="residual")
        total = su.info()["ticks_total"]
        dt_su = _timed_steps(su, total, stream)
        info = su.info()
    print(f"[leg surrogate] exact {ms_exact:.1f} ms per step, surrogate run {dt_su:.2f} s "
          f"({info['surr_ticks']} network ticks)", file=sys.stderr, flush=True)
    # the same run with rechecks: during a fallback every tick is a check too
    with SSM(w, precision=prec, stream=stream) as su:
        su.surrogate_load(master)
        su.surrogate_enable(check_every=every, tol=tol, mode="residual", recheck=True)
        dt_rc = _timed_steps(su, total, stream)
        info_rc = su.info()
    print(f"[leg surrogate] with rechecks {dt_rc:.2f} s ({info_rc['surr_ticks']} network ticks, "
          f"{info_rc['surr_rechecks']} rechecks)", file=sys.stderr, flush=True)
    # fixed rMSE at the reduced size
    g = golden_fixed_rmse("surrogate_reduced")
    wr = W.surrogate_d2(N=g["N"], h=g["h"], h_fine=g["proxy_h"])
    with SSM(W.with_h(wr, g["proxy_h"]), precision="fp64", stream=stream) as r:
        r.run()
        X_ref = r.state(0)
    with SSM(wr, precision=prec, stream=stream) as a:
        a.surrogate_load(master)
        a.surrogate_enable(check_every=every, tol=tol, mode="residual")
        a.run()
        ia = a.info()
        Xa = a.state(0)
    with SSM(wr, precision=prec, stream=stream) as a:
        a.surrogate_load(master)
        a.surrogate_enable(check_every=every, tol=tol, mode="residual", recheck=True)
        a.run()
        ic = a.info()
        Xc = a.state(0)
    with SSM(wr, precision=prec, stream=stream) as b:
        b.run()
        Xb = b.state(0)
    rm = lambda X: math.sqrt(float(np.sum((X - X_ref) ** 2)) / g["N"])
    r_s, r_e, r_c = rm(Xa), rm(Xb), rm(Xc)
    return {
        "workload": f"SSM d=2 N={N} T=1 h=2^-9 Gaussian interaction (l=1), radial cubic v, diagonal sigma; {prec}",
        "training": {"rows": n_rows, "from": "exact runs of ensembles 1-2 at N=2^18, 40 states each "
                                             "(every 2 ticks to tick 32, every 8 to 128, every 32 after)",
                     "rows_seconds": t_data, "adam_steps": int(hist.size), "batch": 4096, "adam_seconds": t_train,
                     "loss_first": float(hist[:50].mean()), "loss_last": float(hist[-200:].mean())},
        "exact": {"ms_per_step": ms_exact, "particle_steps_per_s": N / (ms_exact / 1e3), "timed_steps": n_ex},
        "surrogate": {"rule": f"residual mode, exact check every {every} steps, fallback above {tol:g}",
                      "seconds": dt_su, "steps": total, "particle_steps_per_s": N * total / dt_su,
                      "checks": info["surr_checks"], "network_steps": info["surr_ticks"],
                      "fallback_steps": info["surr_fallback_ticks"], "check_err_last": info["surr_last_err"],
                      "check_err_max": info["surr_max_err"]},
        "speedup_vs_exact": (ms_exact / 1e3 * total) / dt_su,
        "surrogate_recheck": {"rule": f"as above, and during a fallback every tick is a check too "
                                      f"(ssm_surrogate_recheck; an extension of the rule)",
                              "seconds": dt_rc, "particle_steps_per_s": N * total / dt_rc,
                              "checks": info_rc["surr_checks"], "rechecks": info_rc["surr_rechecks"],
                              "network_steps": info_rc["surr_ticks"], "check_err_max": info_rc["surr_max_err"],
                              "speedup_vs_exact": (ms_exact / 1e3 * total) / dt_rc},
        "fixed_rmse": {"workload": g["workload"] + f", proxy h={g['proxy_h']:g} (GPU FP64 run)",
                       "rmse_oracle_exact": g["rmse"], "rmse_gpu_surrogate": r_s, "rmse_gpu_exact_fp32": r_e,
                       "ratio_surrogate_to_oracle": r_s / g["rmse"],
                       "within_5_percent": abs(r_s - g["rmse"]) <= 0.05 * g["rmse"],
                       "network_steps": ia["surr_ticks"], "checks": ia["surr_checks"],
                       "recheck": {"rmse_gpu_surrogate": r_c, "ratio_to_oracle": r_c / g["rmse"],
                                   "within_5_percent": abs(r_c - g["rmse"]) <= 0.05 * g["rmse"],
                                   "network_steps": ic["surr_ticks"], "checks": ic["surr_checks"],
                                   "rechecks": ic["surr_rechecks"]}},
    }


def leg_batched(args, stream) -> dict:
    """The metric's batched leg on the batched case (64 ensembles, N_e
    log-uniform in [2^10, 2^16], h = 2^-4..2^-8 in one context on a 2^-12
    grid, T = 1, FP32-compensated): whole-run throughput with the library's
    default tiling and with the autotuner's choice for this workload, and the
    fixed-rMSE check per step size on a reduced batch (8 ensembles, N_e in
    [2^8, 2^11]) against the oracle's strong errors stored in
    tests/golden/fixed_rmse.json, with the GPU's FP64 2^-12 run as the proxy."""
    import numpy as np
    from paper_2105_09688_amd import workloads as W
    from paper_2105_09688_amd.ssm import SSM
    from paper_2105_09688_amd.tune import autotune
    prec = "fp32_kahan"
    w = W.batched(levels=(4, 5, 6, 7, 8))
    out = {"workload": "64 ensembles, N_e log-uniform in [2^10, 2^16], h=2^-4..2^-8 on a 2^-12 grid, T=1, " + prec}
    runs = {}
    t0 = time.perf_counter()
    tuned = autotune(w, prec, stream=stream, use_cache=False)
    t_tune = time.perf_counter() - t0
    for label, kw in (("default", {}), ("autotuned", {k: tuned[k] for k in
                                                     ("targets_per_lane", "sources_per_item", "pair_scheme")})):
        with SSM(w, precision=prec, stream=stream, **kw) as s:
            i = s.info()
            total = i["ticks_total"]
            dt = _timed_steps(s, total, stream)
        runs[label] = {"seconds": dt, "particle_steps_per_s": particle_steps(w, total) / dt,
                       "targets_per_lane": i["targets_per_lane"], "sources_per_item": i["sources_per_item"],
                       "pair_scheme": i["pair_scheme"], "pair_work_items_phase0": i["n_pair_items"]}
    out.update(runs=runs, autotune_seconds=t_tune, particle_steps=particle_steps(w, total))
    best = max(runs, key=lambda k: runs[k]["particle_steps_per_s"])
    out["particle_steps_per_s"] = runs[best]["particle_steps_per_s"]
    out["tiling_used"] = best
    g = golden_fixed_rmse("batched_reduced")
    levels = tuple(g["levels"])
    wr = W.batched(n_ens=len(g["sizes"]), levels=levels, h_fine=g["proxy_h"], sizes=g["sizes"])
    ref_w = W.with_systems(wr, [(N, e, g["proxy_h"]) for e, N in enumerate(g["sizes"])])
    with SSM(wr, precision=prec, stream=stream) as a, SSM(ref_w, precision="fp64", stream=stream) as r:
        a.run()
        r.run()
        per = {}
        for li, l in enumerate(levels):
            sq, cnt = 0.0, 0
            for e, N in enumerate(g["sizes"]):
                sq += a.sqdiff(e * len(levels) + li, r, e)
                cnt += N
            per[f"2^-{l}"] = math.sqrt(sq / cnt)
    ratios = {k: per[k] / g["rmse"][k] for k in per}
    out["fixed_rmse"] = {"workload": g["workload"] + f", proxy h={g['proxy_h']:g} (GPU FP64 run)",
                         "rmse_oracle": g["rmse"], "rmse_gpu": per, "ratio": ratios,
                         "within_5_percent": all(abs(r - 1.0) <= 0.05 for r in ratios.values())}
    print(f"[leg batched] {out['particle_steps_per_s']:.3e} particle-steps/s ({best}), autotune {t_tune:.1f} s",
          file=sys.stderr, flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=16)
    ap.add_argument("--precision", default="fp32_kahan", choices=["fp64", "fp32", "fp32_kahan"])
    ap.add_argument("--N", type=int, default=0)
    ap.add_argument("--train-steps", type=int, default=64000)
    ap.add_argument("--study", choices=["none", "precision", "batched", "surrogate", "surrogate_tick", "small", "families",
                                        "stability"],
                    default="none",
                    help="run a study of another workload instead of the throughput line")
    ap.add_argument("--legs", default="surrogate,batched",
                    help="the metric's other legs to add to the line: comma-separated subset of "
                         "'surrogate,batched', or 'none'")
    ap.add_argument("--settle-s", type=float, default=1.0,
                    help="seconds of untimed pair-kernel work before the timed context (steady clocks)")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--tune", action="store_true",
                    help="autotune the pair tiling first (default: the library's default tiling, which the "
                         "autotuner also picks for this workload)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="after the run, one plain device copy of this many MiB (calibrates byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(the per-step all-gather of Y* across GPUs is a design note, not code).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2105_09688_amd import workloads as W
    from paper_2105_09688_amd.ssm import SSM

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.study != "none":
        stream = torch.cuda.Stream()
        fn = {"precision": study_precision, "batched": study_batched, "surrogate": study_surrogate,
              "small": study_small, "families": study_families, "stability": study_stability,
              "surrogate_tick": study_surrogate_tick}[args.study]
        print(json.dumps(fn(args, stream)), flush=True)
        return
    w = W.single_gpu_d1(N=args.N or 2 ** 16)
    N, _, h = w["systems"][0]
    d = w["d"]
    total_steps = int(round(w["T"] / h))
    if args.steps < 1 or args.warmup < 0 or args.warmup + args.steps > total_steps:
        raise SystemExit(f"--warmup + --steps must be at most {total_steps} (T/h) and --steps >= 1: the timed "
                         f"steps run in the same context after the warm-up steps")
    legs = [] if args.legs == "none" else [x for x in args.legs.split(",") if x]
    for x in legs:
        if x not in ("surrogate", "batched"):
            raise SystemExit(f"unknown leg {x!r}")

    stream = torch.cuda.Stream()
    tiling = {}
    if args.tune:
        from paper_2105_09688_amd.tune import autotune
        t = autotune(w, args.precision, stream=stream)
        tiling = {k: t[k] for k in ("targets_per_lane", "sources_per_item", "pair_scheme")}
    settle = settle_clocks(SSM, w, args.precision, stream, args.settle_s)
    # the timed context: warm-up steps, then the timed steps
    s = SSM(w, precision=args.precision, stream=stream, **tiling)
    if args.warmup:
        s.step(args.warmup)
    s.sync()
    # HIP events around the pair and update launches of every k-th tick of the
    # timed steps (an event pair costs a few microseconds of stream time per tick)
    every = 8 if args.steps >= 256 else 4 if args.steps >= 64 else 2 if args.steps >= 8 else 1
    s.profile(True, every=every)
    torch.cuda.synchronize()
    ev0, ev1 = _events(stream)
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
        "clock_settle": {"seconds": settle["seconds"], "untimed_steps": settle["ticks"],
                         "note": "untimed steps of other contexts of the same workload before the timed "
                                 "context, so that the timed steps run at steady clocks; the timed context "
                                 "then takes its --warmup steps and the --steps timed ones"},
        "roofline": {
            "bound": "alu",
            "kernel": "k_pair (O(N^2) interaction sums)",
            "achieved": achieved,
            "peak": peak,
            "unit": "TFLOP/s",
            "frac": achieved / peak,
            "traffic": recorded_traffic(f"k_pair {args.precision} d={d} N={N} R={info['targets_per_lane']} "
                                        f"L={info['sources_per_item']} {info['pair_scheme']}"),
            "flop_per_pair": flops_per_pair(d),
            "issue_ceiling": None if args.precision == "fp64" else issue_ceiling_tflops(d, info["pair_scheme"]),
            "frac_of_issue_ceiling": None if args.precision == "fp64" else achieved / issue_ceiling_tflops(d, info["pair_scheme"]),
            "pairs_per_launch": pairs,
            "avg_launch_ms": pair_avg_s * 1e3,
            "launches": info["pair_launches"],
            "launches_timed_every": every,
        },
        "update_kernel_avg_ms": info["update_ms"] / max(1, info["update_launches"]),
        "tiling": {"targets_per_lane": info["targets_per_lane"], "sources_per_item": info["sources_per_item"],
                   "pair_scheme": info["pair_scheme"], "pair_work_items": info["n_pair_items"],
                   "autotuned": bool(args.tune)},
    }
    if not args.no_check and args.precision != "fp64":
        # pathwise agreement of the timed run with the FP64 path after the same steps
        n_chk = args.warmup + args.steps
        with SSM(w, precision="fp64", stream=stream) as ref:
            ref.step(n_chk)
            ref.sync()
            a, b = s.state(0), ref.state(0)
        out["check"] = {"max_pathwise_err_vs_fp64": float(np.max(np.abs(a - b) / np.maximum(1.0, np.abs(b)))),
                        "steps": n_chk}
    s.close()
    if args.calib_copy_mib > 0:
        n = args.calib_copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["calib_copy_bytes"] = {"read": 4 * n, "write": 4 * n}
    if legs:
        out["legs"] = {}
        if "surrogate" in legs:
            out["legs"]["surrogate"] = leg_surrogate(args, stream)
        if "batched" in legs:
            out["legs"]["batched"] = leg_batched(args, stream)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
