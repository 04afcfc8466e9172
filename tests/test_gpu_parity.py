"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances (pathwise, on the same Philox stream): max_i |x_gpu - x_ref| /
max(1, |x_ref|) <= 1e-10 for FP64 and <= 1e-4 for the FP32 modes.
"""
import math
import sys

import numpy as np
import pytest

import errstats
import oracle
from paper_2105_09688_amd import workloads as W

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10
FP32_TOL = 1e-4


def _say(msg):
    print(f"[gpu-parity] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    return torch


def _err(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.max(np.abs(got - ref) / np.maximum(1.0, np.abs(ref)))) if ref.size else 0.0


def _ssm(w, precision="fp64", **kw):
    from paper_2105_09688_amd.ssm import SSM
    return SSM(w, precision=precision, **kw)


# --------------------------------------------------------------------------- random numbers
def test_philox_blocks_bitwise(torch_cuda):
    from paper_2105_09688_amd.ssm import philox_blocks
    rng = np.random.default_rng(1)
    for _ in range(4):
        ctr = [int(v) for v in rng.integers(0, 2 ** 63, 4)]
        key = [int(v) for v in rng.integers(0, 2 ** 63, 2)]
        _say(f"philox ctr={ctr} key={key}")
        got = philox_blocks(ctr, key, 257).cpu().numpy().view(np.uint64)
        for q in range(0, 257, 16):
            ref = oracle.philox4x64_10([ctr[0] + q, ctr[1], ctr[2], ctr[3]], key)
            assert np.array_equal(got[q], ref), q


@pytest.mark.parametrize("d,r", [(1, 3), (1, 16), (2, 1), (3, 1), (3, 5), (4, 2)])
def test_brownian_increments_match_oracle(torch_cuda, d, r):
    from paper_2105_09688_amd.ssm import brownian
    N, seed, ens, n0, hf = 300, 7, 5, 17, 2.0 ** -10
    _say(f"brownian d={d} r={r}")
    got = brownian(d, N, seed, ens, n0, r, hf).cpu().numpy()
    ref = np.stack([oracle.brownian(seed, d, i, ens, n0, r, hf) for i in range(N)], axis=1)
    err = np.max(np.abs(got - ref))
    _say(f"  max abs diff {err:.3e} (increments up to {np.max(np.abs(ref)):.2f})")
    # a few ulps of the largest increment: the device's own log and sine/cosine
    # against the oracle's libm (measured: at most 1.1e-16 on increments up to 0.3)
    assert err <= 8 * 2.0 ** -52 * np.max(np.abs(ref))


@pytest.mark.parametrize("d,r,prec", [(1, 16, "fp32_kahan"), (2, 16, "fp32"), (3, 4, "fp32_kahan"), (2, 16, "fp64")])
def test_context_increments_match_oracle(torch_cuda, d, r, prec):
    """The increments a context draws, seen through a pure Brownian motion
    (v = 0, b = 0, sigma = 1, X_0 = 0, so X_n = dW_0 + ... + dW_{n-1}), after
    5 steps of r fine increments, against the oracle's increments.  FP32
    modes draw their normals with the FP32 transform: within 1e-6 of the
    largest |X| (the transform's own error plus five roundings of the FP32
    state; measured at most 2.3e-7 of it); FP64 within 8 ulps."""
    N, hf = 2500, 2.0 ** -12
    h = r * hf
    w = dict(d=d, T=8 * h, seed=3, h_fine=hf, systems=[(N, 4, h)],
             v=dict(rho=0.0, a=0.0, kappa=0.0, lam=0.0), b=dict(c0=0.0, lam=0.0, g=0.0, ell=1.0),
             sigma=dict(s0=[1.0] * d, s1=[0.0] * d, s2=[0.0] * d), x0_mean=[0.0] * d, x0_std=[0.0] * d)
    with _ssm(w, prec) as s:
        s.step(5)
        got = s.state(0)
    ref = np.zeros((d, N))
    for i in range(N):
        ref[:, i] = sum(oracle.brownian(w["seed"], d, i, 4, n * r, r, hf) for n in range(5))
    err = float(np.max(np.abs(got - ref)))
    scale = float(np.max(np.abs(ref)))
    _say(f"context increments d={d} r={r} {prec}: max abs diff {err:.3e} (|X| up to {scale:.3f})")
    assert err <= (8 * 2.0 ** -52 if prec == "fp64" else 1e-6) * scale


# --------------------------------------------------------------------------- implicit step (2.3)
@pytest.mark.parametrize("d", [1, 2, 3, 4])
def test_implicit_solve_matches_oracle(torch_cuda, d):
    from paper_2105_09688_amd.ssm import implicit_solve
    torch = torch_cuda
    rng = np.random.default_rng(d)
    N = 2000
    X = rng.normal(size=(d, N)) * 4.0
    X[:, 0] = 0.0
    X[:, 1] = 1e-300
    for (h, rho, a, kappa, lam) in [(2.0 ** -4, 0.0, 1.0, 0.0, 0.0), (2.0 ** -10, 0.0, 1.0, 0.0, 0.0),
                                    (0.05, 2.0, 0.25, 0.0, 0.0), (0.1, -1.0, 0.0, 0.0, 0.0),
                                    (0.01, 0.5, 1.0, 0.3, 0.7)]:
        xbar = rng.normal(size=d)
        m2 = 1.7
        _say(f"implicit d={d} h={h} rho={rho} a={a} kappa={kappa} lam={lam}")
        Y, it = implicit_solve(torch.tensor(X, device="cuda"), h, rho, a, kappa, lam, xbar, m2)
        Y = Y.cpu().numpy()
        it = it.cpu().numpy()
        assert np.all(it >= 0)
        ref = np.stack([oracle.implicit(X[:, i], h, rho, a, kappa, lam, xbar, m2)[0] for i in range(N)], axis=1)
        assert np.max(np.abs(Y - ref) / np.maximum(1e-300, np.abs(ref)).clip(min=1.0)) <= 1e-14


# --------------------------------------------------------------------------- pairwise sums (2.4)
@pytest.mark.parametrize("d,ell", [(1, 1.0), (2, 1.0), (3, 0.5), (4, 0.7)])
@pytest.mark.parametrize("N", [1, 2, 63, 64, 65, 257, 1000, 4099])
def test_pair_sum_matches_oracle(torch_cuda, d, ell, N):
    from paper_2105_09688_amd.ssm import pair_sum
    torch = torch_cuda
    Y = W.random_cloud(d, N, seed=N + 10 * d, loc=0.3, scale=1.5)
    ref = oracle.pair_sum(Y, ell)
    _say(f"pair_sum fp64 d={d} N={N}")
    got = pair_sum(torch.tensor(Y, device="cuda"), ell, "fp64").cpu().numpy()
    assert _err(got, ref) <= 1e-12
    for prec in ("fp32", "fp32_kahan"):
        _say(f"pair_sum {prec} d={d} N={N}")
        Y32 = np.asarray(Y, dtype=np.float32)  # the same rounded inputs on both sides
        got = pair_sum(torch.tensor(Y32, device="cuda"), ell, prec).cpu().numpy()
        ref32 = oracle.pair_sum(Y32.astype(np.float64), ell)
        assert _err(got, ref32) <= 2e-6, prec


def test_pair_sum_full_size_sampled_and_zero_net_force(torch_cuda):
    """N = 2^16 (the single-GPU d=1 size) and N = 2^18 at d=3: sampled targets
    against the oracle, plus sum_i K^i = 0 (odd kernel) over all targets."""
    from paper_2105_09688_amd.ssm import pair_sum
    torch = torch_cuda
    rng = np.random.default_rng(3)
    for d, N, ell in [(1, 2 ** 16, 1.0), (3, 2 ** 18, 0.5)]:
        Y = W.random_cloud(d, N, seed=77 + d)
        idx = np.sort(rng.choice(N, 96, replace=False))
        idx[-1] = N - 1
        ref = oracle.pair_sum_at(Y, ell, idx)
        for prec, tol in (("fp64", 1e-12), ("fp32_kahan", 2e-6), ("fp32", 2e-6)):
            _say(f"pair_sum full size d={d} N={N} {prec}")
            Yh = np.asarray(Y, dtype=np.float64 if prec == "fp64" else np.float32)
            K = pair_sum(torch.tensor(Yh, device="cuda"), ell, prec).cpu().numpy()
            r = ref if prec == "fp64" else oracle.pair_sum_at(Yh.astype(np.float64), ell, idx)
            assert _err(K[:, idx], r) <= tol, prec
            net = np.abs(K.sum(axis=1))
            assert np.all(net <= (1e-9 if prec == "fp64" else 1e-3) * np.abs(K).sum(axis=1)), (prec, net)


def test_full_size_single_gpu_steps_match_oracle(torch_cuda):
    """The single-GPU d = 1 workload at full size (N = 2^16, h = 2^-10) in the
    tiling the benchmark times (library default: symmetric scheme, 4 targets
    per lane, 320 sources per item): the first two steps against the oracle's
    own steps from its X_0, pathwise, in FP32-compensated and FP64."""
    w = W.single_gpu_d1()
    N, ens, h = w["systems"][0]
    X = oracle.init_state(w, ens, N)
    refs = []
    for n in range(2):
        _say(f"oracle full-size step {n}")
        X, _ = oracle.step(w, ens, h, n, X)
        refs.append(X)
    for prec, tol in (("fp32_kahan", FP32_TOL), ("fp64", FP64_TOL)):
        with _ssm(w, prec) as s:
            info = s.info()
            if prec == "fp32_kahan":
                assert (info["pair_scheme"], info["targets_per_lane"], info["sources_per_item"]) == ("symmetric", 4, 320)
            for n in range(2):
                _say(f"gpu full-size step {n} {prec}")
                s.step(1)
                err = _err(s.state(0), refs[n])
                _say(f"  max rel err {err:.3e}")
                assert err <= tol, (prec, n, err)


def _sample(N, k, seed):
    idx = np.sort(np.random.default_rng(seed).choice(N, k, replace=False))
    idx[0], idx[-1] = 0, N - 1
    return idx


@pytest.mark.parametrize("case", ["precision_d3_N2^18", "surrogate_d2_N2^20"])
def test_full_size_first_step_sampled(torch_cuda, case):
    """The d = 3 precision case (N = 2^18) and the d = 2 surrogate case
    (N = 2^20) at full size in the library's default tiling: the first exact
    step at 256 sampled particles against the oracle's step evaluated there
    (its own X_0; Y* solved for every particle), FP32-compensated and FP64."""
    w = W.precision_d3() if case.startswith("precision") else W.surrogate_d2()
    N, ens, h = w["systems"][0]
    idx = _sample(N, 256, 11)
    _say(f"oracle step at 256 particles, {case}")
    ref = oracle.step_at(w, ens, h, 0, oracle.init_state(w, ens, N), idx)
    for prec, tol in (("fp32_kahan", FP32_TOL), ("fp64", FP64_TOL)):
        _say(f"gpu first step {case} {prec}")
        with _ssm(w, prec) as s:
            s.step(1)
            err = _err(s.state(0)[:, idx], ref)
        _say(f"  max rel err {err:.3e}")
        assert err <= tol, (case, prec, err)


def test_maximum_size_symmetric_step_sampled(torch_cuda):
    """d = 2, N = 2^22 (four times the surrogate case) in the symmetric
    scheme: its 8192 target groups would need 256 GiB of j-side rows (more
    than 40 % of the free device memory), so the library runs them in bands
    of 512 groups (16 GiB, k_jfold).  The first exact step at 128 sampled particles against the
    oracle's step there, FP32-compensated."""
    w = W.surrogate_d2(N=2 ** 22)
    N, ens, h = w["systems"][0]
    idx = _sample(N, 128, 21)
    _say("oracle step at 128 particles, d=2 N=2^22")
    ref = oracle.step_at(w, ens, h, 0, oracle.init_state(w, ens, N), idx)
    with _ssm(w, "fp32_kahan") as s:
        info = s.info()
        _say(f"d=2 N=2^22: {info['pair_scheme']}, bands of {info['jside_band_groups']} groups, "
             f"{info['device_bytes'] / 2 ** 30:.1f} GiB")
        assert info["pair_scheme"] == "symmetric" and info["jside_band_groups"] == 512
        assert info["device_bytes"] < 20 * 2 ** 30
        s.step(1)
        err = _err(s.state(0)[:, idx], ref)
    _say(f"  max rel err {err:.3e}")
    assert err <= FP32_TOL


def _banded_case(d):
    """Three systems of ragged sizes (6, 3 and 2 target groups of 256 at one
    target per lane) with the coefficients of the workload of that d."""
    base = {1: W.small_parity(n_ens=1, N=8, h=2.0 ** -6, h_fine=2.0 ** -6),
            2: W.surrogate_d2(N=8, h=2.0 ** -6, h_fine=2.0 ** -6),
            3: W.precision_d3(N=8, h=2.0 ** -6)}[d]
    w = W.with_systems(base, [(1500, 0, 2.0 ** -6), (700, 1, 2.0 ** -6), (300, 2, 2.0 ** -6)])
    w["T"] = 4 * 2.0 ** -6
    return w


@pytest.mark.parametrize("d,prec", [(1, "fp64"), (1, "fp32_kahan"), (2, "fp32_kahan"), (3, "fp64")])
def test_banded_jside_matches_oracle_and_unbanded(torch_cuda, d, prec):
    """The symmetric scheme with its j-side rows in bands of 1, 2 and 4
    target groups (forced; the fold adds each band's rows to a running total
    per particle) against the oracle (FP64 1e-10, FP32 1e-4), against the
    unbanded run (summation order only: FP64 1e-13, FP32 1e-6), and bitwise
    reproducible."""
    w = _banded_case(d)
    ref = oracle.run(w)
    tol = FP64_TOL if prec == "fp64" else FP32_TOL
    with _ssm(w, prec, targets_per_lane=1, pair_scheme="symmetric") as u:
        u.run()
        assert u.info()["jside_band_groups"] == 0
        plain = u.states()
    for band in (1, 2, 4):
        runs = []
        for rep in range(2 if band == 2 else 1):
            with _ssm(w, prec, targets_per_lane=1, pair_scheme="symmetric", jside_band_groups=band) as b:
                assert b.info()["jside_band_groups"] == band
                b.run()
                runs.append(b.states())
        got = runs[0]
        e_or = max(_err(g, r) for g, r in zip(got, ref))
        e_un = max(_err(g, r) for g, r in zip(got, plain))
        _say(f"banded j-side d={d} {prec} band={band}: vs oracle {e_or:.3e}, vs unbanded {e_un:.3e}")
        assert e_or <= tol
        assert e_un <= (1e-13 if prec == "fp64" else 1e-6)
        if len(runs) == 2:
            assert all(np.array_equal(a, b) for a, b in zip(runs[0], runs[1]))


def test_full_size_batched_first_tick_sampled(torch_cuda):
    """The batched case at full size (64 ensembles, N_e in [2^10, 2^16], five
    step sizes, one context, shared Brownian windows): after the first tick,
    on which every system steps, sampled particles of the largest and the
    smallest ensemble at every step size against the oracle's step of that
    system alone."""
    w = W.batched(levels=(4, 5, 6, 7, 8))
    systems = w["systems"]
    sizes = sorted({sy[0] for sy in systems})
    pick = [k for k, sy in enumerate(systems) if sy[0] in (sizes[0], sizes[-1])]
    with _ssm(w, "fp32_kahan") as s:
        s.step(1)
        got = {k: s.state(k) for k in pick}
    for k in pick:
        N, ens, h = systems[k]
        idx = _sample(N, 64, k)
        _say(f"batched system {k}: N={N} ens={ens} h={h}")
        ref = oracle.step_at(w, ens, h, 0, oracle.init_state(w, ens, N), idx)
        assert _err(got[k][:, idx], ref) <= FP32_TOL, (k, N, h)


# --------------------------------------------------------------------------- whole runs
@pytest.fixture(scope="module")
def c0_oracle():
    w = W.small_parity()
    _say("oracle run: 10 x 1000 particles, 256 steps")
    return w, oracle.run(w)


def test_run_small_parity_fp64(torch_cuda, c0_oracle):
    w, ref = c0_oracle
    _say("gpu fp64 run 10 x 1000 x 256 steps")
    with _ssm(w, "fp64") as s:
        s.run()
        got = s.states()
        for e in range(len(ref)):
            assert _err(got[e], ref[e]) <= FP64_TOL, e
            m, v = s.moments(e)
            mr, vr = oracle.moments(ref[e])
            assert np.allclose(m, mr, rtol=0, atol=1e-10) and np.allclose(v, vr, rtol=0, atol=1e-10)
        info = s.info()
        assert info["newton_failures"] == 0 and info["nonfinite"] == 0 and info["tick"] == 256


@pytest.mark.parametrize("precision", ["fp32", "fp32_kahan"])
def test_run_small_parity_fp32(torch_cuda, c0_oracle, precision):
    w, ref = c0_oracle
    _say(f"gpu {precision} run 10 x 1000 x 256 steps")
    with _ssm(w, precision) as s:
        s.run()
        got = s.states()
    errs = [_err(g, r) for g, r in zip(got, ref)]
    _say(f"{precision} max pathwise error {max(errs):.3e}")
    assert max(errs) <= FP32_TOL


def test_stepwise_parity_and_implicit_state(torch_cuda):
    """Step by step on one system: X_n and the implicit state Y*_n = F_h(X_n)
    against the oracle's own step-by-step run from its X_0."""
    w = W.small_parity(n_ens=1, N=777, h=2.0 ** -6, h_fine=2.0 ** -8)
    h = 2.0 ** -6
    with _ssm(w, "fp64") as s:
        X = oracle.init_state(w, 0, 777)
        assert _err(s.state(0, "x"), X) <= 1e-15
        for n in range(8):
            _say(f"stepwise n={n}")
            X_next, Y_ref = oracle.step(w, 0, h, n, X)
            assert _err(s.state(0, "y"), Y_ref) <= 1e-13
            s.step(1)
            assert _err(s.state(0, "x"), X_next) <= 1e-13
            X = X_next


def test_multilevel_batched_equals_separate_runs(torch_cuda):
    """Uneven ensembles at several step sizes in one context == each system run
    alone by the oracle (same Brownian paths per ensemble)."""
    sizes = [300, 1000, 65, 1]
    w = W.batched(n_ens=4, levels=(4, 5, 6), h_fine=2.0 ** -8, sizes=sizes)
    w["T"] = 0.25
    _say("oracle: 12 systems")
    ref = oracle.run(w)
    for prec, tol in (("fp64", FP64_TOL), ("fp32_kahan", FP32_TOL)):
        _say(f"gpu batched {prec}")
        with _ssm(w, prec) as s:
            s.run()
            got = s.states()
        for k, (g, r) in enumerate(zip(got, ref)):
            assert _err(g, r) <= tol, (prec, k, w["systems"][k])


@pytest.mark.parametrize("d", [2, 3])
def test_shared_brownian_windows_in_d_2_and_3(torch_cuda, d):
    """Path groups (one ensemble and size at several step sizes) sharing a
    Brownian window, in d = 2 (8 normals per tick) and d = 3 with h_fine =
    h_min (3 normals per tick, so Philox blocks straddle ticks), beside a
    system of its own: every system equals the oracle's run of it alone."""
    if d == 2:
        base = W.surrogate_d2(N=300, h=2.0 ** -6, h_fine=2.0 ** -8)
        hs = (2.0 ** -4, 2.0 ** -5, 2.0 ** -6)
    else:
        base = W.precision_d3(N=300, h=2.0 ** -6)
        hs = (2.0 ** -3, 2.0 ** -4, 2.0 ** -6)
    systems = [(300, 0, h) for h in hs] + [(65, 1, hs[0]), (65, 1, hs[2]), (129, 2, hs[1])]
    w = W.with_systems(base, systems)
    w["T"] = 0.25
    _say(f"oracle: {len(systems)} systems, d={d}")
    ref = oracle.run(w)
    for prec, tol in (("fp64", FP64_TOL), ("fp32_kahan", FP32_TOL)):
        _say(f"gpu windows d={d} {prec}")
        with _ssm(w, prec) as s:
            s.run()
            got = s.states()
        for k, (g, r) in enumerate(zip(got, ref)):
            assert _err(g, r) <= tol, (prec, k, systems[k])


@pytest.mark.parametrize("precision,tol", [("fp64", FP64_TOL), ("fp32_kahan", FP32_TOL), ("fp32", FP32_TOL)])
def test_run_d3_and_d2(torch_cuda, precision, tol):
    for w in (W.precision_d3(N=700), W.surrogate_d2(N=900, h=2.0 ** -9, h_fine=2.0 ** -10)):
        w["T"] = 2.0 ** -4
        _say(f"d={w['d']} {precision}")
        ref = oracle.run(w)[0]
        with _ssm(w, precision) as s:
            s.run()
            got = s.state(0)
        assert _err(got, ref) <= tol


def test_run_d4_in_both_schemes(torch_cuda):
    """d = 4, the largest dimension the library takes: radial cubic drift,
    Gaussian interaction, diagonal affine noise, a ragged N, in FP64 and
    FP32-compensated, symmetric (R = 1, and R = 2 in FP32, where a group of
    512 x 4 fills the float row) and ordered, against the oracle pathwise."""
    w = W.precision_d3(N=601, h=2.0 ** -8)
    w.update(d=4, T=2.0 ** -4, x0_mean=[0.2, -0.1, 0.0, 0.3], x0_std=[0.8, 1.0, 0.6, 0.9],
             sigma=dict(s0=[0.2, 0.25, 0.15, 0.3], s1=[0.1, 0.0, 0.05, 0.1], s2=[0.0, 0.1, 0.0, 0.0]))
    w["b"]["ell"] = 0.7
    ref = oracle.run(w)[0]
    cases = [("fp64", FP64_TOL, "symmetric", 1), ("fp64", FP64_TOL, "ordered", 2),
             ("fp32_kahan", FP32_TOL, "symmetric", 1), ("fp32_kahan", FP32_TOL, "symmetric", 2),
             ("fp32_kahan", FP32_TOL, "ordered", 4)]
    for prec, tol, scheme, R in cases:
        _say(f"d=4 {prec} {scheme} R={R}")
        with _ssm(w, prec, pair_scheme=scheme, targets_per_lane=R) as s:
            assert s.info()["pair_scheme"] == scheme
            s.run()
            assert _err(s.state(0), ref) <= tol, (prec, scheme, R)


def test_measure_dependent_v_unfused_path(torch_cuda):
    """v depends on mu^X (mean and second moment): the implicit solve runs in
    its own kernel after the moments of the new cloud are reduced."""
    w = W.small_parity(n_ens=2, N=513, h=2.0 ** -6, h_fine=2.0 ** -6)
    w["T"] = 0.25
    w["v"] = dict(rho=-1.0, a=0.5, kappa=0.3, lam=0.5)
    w["b"] = dict(c0=0.2, lam=0.4, g=0.7, ell=0.8)
    w["sigma"] = dict(s0=[0.1], s1=[0.3], s2=[0.2])
    ref = oracle.run(w)
    _say("gpu unfused fp64")
    with _ssm(w, "fp64") as s:
        s.run()
        got = s.states()
    for g, r in zip(got, ref):
        assert _err(g, r) <= FP64_TOL


def test_linear_ou_without_pair_term(torch_cuda):
    w = W.ou(rho=-0.7, lam=0.4, eta=0.5, x0=1.0, x0_std=0.2, N=4097, h=2.0 ** -7, n_ens=2, T=0.5)
    ref = oracle.run(w)
    with _ssm(w, "fp64") as s:
        s.run()
        for e in range(2):
            assert _err(s.state(e), ref[e]) <= FP64_TOL


def test_bound_state_is_the_context_state(torch_cuda):
    """A torch tensor bound as the state X (ssm_bind_state): the run in it
    equals an unbound run bitwise and its views equal get_state; X written
    through the tensor followed by ssm_state_refresh equals ssm_set_state of
    the same values; undersized or misaligned buffers are refused."""
    import ctypes as C
    from paper_2105_09688_amd import _lib
    torch = torch_cuda
    w = W.batched(n_ens=2, levels=(4, 5), h_fine=2.0 ** -8, sizes=[300, 65])
    w["T"] = 0.25
    for prec in ("fp64", "fp32_kahan"):
        _say(f"bound state {prec}")
        with _ssm(w, prec) as a, _ssm(w, prec) as b:
            buf = a.bind_state()
            P, offs, e = a.state_layout()
            assert tuple(buf.shape) == (w["d"], P) and all(o % 256 == 0 for o in offs)
            assert e == (8 if prec == "fp64" else 4)
            a.step(3)
            b.step(3)
            a.sync()
            b.sync()
            for s in range(len(a.N)):
                va = a.state_view(s).double().cpu().numpy()
                assert np.array_equal(va, a.state(s)) and np.array_equal(va, b.state(s)), (prec, s)
            Xn = np.random.default_rng(5).normal(size=(w["d"], a.N[0]))
            Xs = Xn.astype(np.float64 if prec == "fp64" else np.float32)
            a.state_view(0).copy_(torch.tensor(Xs, device="cuda"))
            torch.cuda.synchronize()
            a.refresh(0)
            b.set_state(0, Xs.astype(np.float64))
            a.step(2)
            b.step(2)
            for s in range(len(a.N)):
                assert np.array_equal(a.state(s), b.state(s)), (prec, s)
                assert np.array_equal(a.state(s, "y"), b.state(s, "y")), (prec, s)
    with _ssm(w, "fp64") as c:
        P, _, e = c.state_layout()
        t = torch.zeros(w["d"] * P + 8, dtype=torch.float64, device="cuda")
        lib = _lib.load()
        assert lib.ssm_bind_state(c._h, C.c_void_p(t.data_ptr()), w["d"] * P * e - 8) == _lib.SSM_ERR_INVALID
        assert lib.ssm_bind_state(c._h, C.c_void_p(t.data_ptr() + 8), w["d"] * P * e) == _lib.SSM_ERR_INVALID
        assert lib.ssm_state_refresh(c._h, 7) == _lib.SSM_ERR_INVALID


def test_single_particle_and_ragged_sizes(torch_cuda):
    for N in (1, 2, 255, 257):
        w = W.small_parity(n_ens=1, N=N, h=2.0 ** -5, h_fine=2.0 ** -5)
        w["T"] = 2.0 ** -3
        ref = oracle.run(w)[0]
        with _ssm(w, "fp64") as s:
            s.run()
            assert _err(s.state(0), ref) <= FP64_TOL, N


def test_determinism_bitwise(torch_cuda):
    w = W.small_parity(n_ens=3, N=1500)
    w["T"] = 2.0 ** -4
    outs = []
    for _ in range(2):
        with _ssm(w, "fp32_kahan") as s:
            s.run()
            outs.append(s.states())
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


def test_tiling_does_not_change_results_beyond_rounding(torch_cuda):
    w = W.small_parity(n_ens=2, N=3000)
    w["T"] = 2.0 ** -5
    base = None
    for R, L in ((1, 64), (2, 512), (4, 0), (8, 1000)):
        _say(f"tiling R={R} L={L}")
        with _ssm(w, "fp64", targets_per_lane=R, sources_per_item=L) as s:
            s.run()
            got = s.states()
        if base is None:
            base = got
        for g, b in zip(got, base):
            assert _err(g, b) <= 1e-12


def test_rmse_matches_oracle_within_5_percent(torch_cuda):
    """The strong error of a run at h against its proxy at h_ref (Section 3),
    GPU vs oracle: the 'fixed rMSE' criterion (within 5 %)."""
    base = W.small_parity(n_ens=4, N=500, h_fine=2.0 ** -12)
    ref_w = W.with_h(base, 2.0 ** -12)
    _say("oracle reference run at 2^-12")
    ref = oracle.run(ref_w)
    for h in (2.0 ** -6, 2.0 ** -8):
        oh = oracle.run(W.with_h(base, h))
        r_or = oracle.strong_error(oh, ref)
        for prec in ("fp64", "fp32_kahan"):
            _say(f"rmse h={h} {prec}")
            with _ssm(W.with_h(base, h), prec) as a, _ssm(ref_w, prec) as b:
                a.run()
                b.run()
                r_gpu, per = a.rmse(b)
                sa, sb = a.states(), b.states()
            # the device reduction equals the host formula on the same states
            assert r_gpu == pytest.approx(errstats.strong_error(sa, sb), rel=1e-12)
            assert abs(r_gpu - r_or) <= 0.05 * r_or, (prec, h, r_gpu, r_or)
            if prec == "fp64":
                assert abs(r_gpu - r_or) <= 1e-8 * r_or


def test_errors_are_reported(torch_cuda):
    from paper_2105_09688_amd import SSMError
    w = W.small_parity(n_ens=1, N=100)
    w["T"] = 2.0 ** -6
    with _ssm(w, "fp64") as s:
        s.run()
        with pytest.raises(SSMError) as e:
            s.step(1)
        assert e.value.status == -6
    w["newton_max_iter"] = 1
    w["x0_std"] = [20.0]
    with pytest.raises(SSMError) as e:
        with _ssm(w, "fp64") as s:
            s.run()
    assert e.value.status == -2


def test_batched_levels_rmse_match_oracle_within_5_percent(torch_cuda):
    """Reduced batched case (uneven ensembles x three step sizes in one FP32
    context): per-level strong error against a 2^-10 proxy on the same paths
    matches the oracle's within 5 %, and the per-system sqdiff entry point
    agrees with the host formula."""
    import math
    sizes = [64, 300, 129, 512, 1000, 77]
    levels = (4, 5, 6)
    w = W.batched(n_ens=len(sizes), levels=levels, h_fine=2.0 ** -10, sizes=sizes)
    ref_w = W.with_systems(w, [(N, e, 2.0 ** -10) for e, N in enumerate(sizes)])
    _say("oracle batched + reference")
    o = oracle.run(w)
    o_ref = oracle.run(ref_w)
    with _ssm(w, "fp32_kahan") as a, _ssm(ref_w, "fp32_kahan") as b:
        a.run()
        b.run()
        for li, l in enumerate(levels):
            sq_g = sq_o = 0.0
            cnt = 0
            for e, N in enumerate(sizes):
                k = e * len(levels) + li
                assert w["systems"][k] == (N, e, 2.0 ** -l)
                g = a.sqdiff(k, b, e)
                host = float(np.sum((a.state(k) - b.state(e)) ** 2))
                assert g == pytest.approx(host, rel=1e-12, abs=1e-300)
                sq_g += g
                sq_o += float(np.sum((o[k] - o_ref[e]) ** 2))
                cnt += N
            r_g, r_o = math.sqrt(sq_g / cnt), math.sqrt(sq_o / cnt)
            _say(f"level 2^-{l}: rmse gpu {r_g:.6e} oracle {r_o:.6e}")
            assert abs(r_g - r_o) <= 0.05 * r_o


def test_graph_replays_match_eager_bitwise(torch_cuda):
    """Each tick phase's captured graph is replayed many times, with eager work
    (state copies, moments) and synchronizations between replays; every
    checked state equals the eager run's bitwise."""
    sizes = [300, 1000, 65]
    w = W.batched(n_ens=3, levels=(4, 5, 6), h_fine=2.0 ** -8, sizes=sizes)
    w["T"] = 0.5
    # the multi-launch path both times (graph replays never run the persistent path)
    with _ssm(w, "fp32_kahan", persistent=-1) as eager, _ssm(w, "fp32_kahan", graphs=True) as g:
        ticks = eager.info()["ticks_total"]
        for t in range(ticks):
            eager.step(1)
            g.step(1)
            if t % 5 == 0 or t == ticks - 1:
                _say(f"graph replay tick {t}")
                for k in range(len(w["systems"])):
                    assert np.array_equal(eager.state(k), g.state(k)), (t, k)
                    assert np.array_equal(eager.state(k, "y"), g.state(k, "y")), (t, k)
                m1, _ = eager.moments(0)
                m2, _ = g.moments(0)
                assert np.array_equal(m1, m2)
        assert g.info()["tick"] == ticks
    # one long graph-mode run equals the oracle
    w2 = W.small_parity(n_ens=2, N=700)
    w2["T"] = 2.0 ** -3
    ref = oracle.run(w2)
    with _ssm(w2, "fp64", graphs=True) as s:
        s.run()
        for e in range(2):
            assert _err(s.state(e), ref[e]) <= FP64_TOL


def test_symmetric_and_ordered_schemes_agree(torch_cuda):
    """The symmetric pair scheme (each unordered pair once, +q / -q) and the
    ordered one give the same FP32 runs up to summation rounding, for every
    dimension, for ragged sizes and across several target-block sizes."""
    for w in (W.small_parity(n_ens=2, N=1500), W.precision_d3(N=777), W.surrogate_d2(N=1300, h_fine=2.0 ** -9)):
        w["T"] = 2.0 ** -5 if w["d"] == 1 else 2.0 ** -6
        base = None
        Rmax = {1: 8, 2: 4, 3: 2}[w["d"]]  # a symmetric target group's j-side must fit LDS
        for scheme, R, L in (("ordered", 2, 0), ("symmetric", 1, 64), ("symmetric", 2, 0), ("symmetric", Rmax, 272)):
            _say(f"scheme d={w['d']} {scheme} R={R} L={L}")
            with _ssm(w, "fp32_kahan", pair_scheme=scheme, targets_per_lane=R, sources_per_item=L) as s:
                s.run()
                got = s.states()
                assert s.info()["pair_scheme"] == scheme
            if base is None:
                base = got
            for g, b in zip(got, base):
                assert _err(g, b) <= 2e-6


def test_symmetric_fp64_matches_oracle_for_every_fitting_tiling(torch_cuda):
    """FP64 in both pair schemes against the oracle, pathwise: the symmetric
    scheme at every target-block size whose group fits the double LDS row
    (R x d <= 4; R = 2 at d = 3), with the default source range and one
    that is 16 past the row's capacity (two LDS pieces per item), on ragged
    sizes in d = 1, 2, 3."""
    for w in (W.small_parity(n_ens=2, N=1500), W.precision_d3(N=777), W.surrogate_d2(N=1300, h_fine=2.0 ** -9)):
        w["T"] = 2.0 ** -5 if w["d"] == 1 else 2.0 ** -6
        _say(f"oracle d={w['d']}")
        ref = oracle.run(w)
        Rs = {1: (1, 2, 4), 2: (1, 2), 3: (1, 2)}[w["d"]]
        past = {1: 1040, 2: 528, 3: 528}[w["d"]]  # 1024 / d doubles per source (1536 / 3 at d = 3), + 16
        cases = [("ordered", 2, 0)] + [("symmetric", R, L) for R in Rs for L in (0, past)]
        for scheme, R, L in cases:
            _say(f"fp64 d={w['d']} {scheme} R={R} L={L}")
            with _ssm(w, "fp64", pair_scheme=scheme, targets_per_lane=R, sources_per_item=L) as s:
                assert s.info()["pair_scheme"] == scheme
                s.run()
                for e, r in enumerate(ref):
                    assert _err(s.state(e), r) <= FP64_TOL, (w["d"], scheme, R, L, e)


def test_per_pair_compensation_matches_oracle(torch_cuda):
    """FP32-compensated with every pair term compensated (kahan_span = 1, the
    precision study's variant, ordered pairs) against the oracle, pathwise,
    and against the default compensated run, in d = 1 and 3 on ragged sizes
    and several target-block sizes."""
    for w in (W.small_parity(n_ens=2, N=1500), W.precision_d3(N=777)):
        w["T"] = 2.0 ** -5 if w["d"] == 1 else 2.0 ** -6
        ref = oracle.run(w)
        with _ssm(w, "fp32_kahan") as s:
            s.run()
            base = s.states()
        for R in (1, 2, 8):
            _say(f"per-pair compensation d={w['d']} R={R}")
            with _ssm(w, "fp32_kahan", kahan_span=1, targets_per_lane=R) as s:
                assert s.info()["pair_scheme"] == "ordered"
                s.run()
                for e, r in enumerate(ref):
                    assert _err(s.state(e), r) <= FP32_TOL, (w["d"], R, e)
                    assert _err(s.state(e), base[e]) <= 2e-6, (w["d"], R, e)


def test_autotuner_choice_is_valid_and_cached(torch_cuda, tmp_path, monkeypatch):
    from paper_2105_09688_amd.tune import autotune
    monkeypatch.setenv("SSM_TUNE_CACHE", str(tmp_path / "tune.json"))
    w = W.single_gpu_d1(N=4096)
    choice = autotune(w, "fp32_kahan", steps=2)
    assert choice["pair_scheme"] in ("symmetric", "ordered") and choice["targets_per_lane"] in (1, 2, 4, 8)
    assert (tmp_path / "tune.json").exists()
    assert autotune(w, "fp32_kahan") == choice  # from the cache
    ref = oracle.run(W.with_systems(w, [(4096, 0, 2.0 ** -10)]), stop_after=8)[0]
    with _ssm(w, "fp32_kahan", targets_per_lane=choice["targets_per_lane"],
              sources_per_item=choice["sources_per_item"], pair_scheme=choice["pair_scheme"]) as s:
        s.step(8)
        assert _err(s.state(0), ref) <= FP32_TOL


def test_autotuner_in_fp64_tries_both_schemes_and_its_choice_matches_oracle(torch_cuda, tmp_path, monkeypatch):
    """The FP64 candidates include the symmetric scheme at every target-block
    size whose group fits the double LDS row; the chosen tiling runs to the
    FP64 bar against the oracle."""
    from paper_2105_09688_amd.tune import autotune, candidates
    cands = candidates(2, "fp64")
    assert {c["pair_scheme"] for c in cands} == {"symmetric", "ordered"}
    assert {c["targets_per_lane"] for c in cands if c["pair_scheme"] == "symmetric"} == {1, 2}
    monkeypatch.setenv("SSM_TUNE_CACHE", str(tmp_path / "tune.json"))
    w = W.surrogate_d2(N=1500, h=2.0 ** -9, h_fine=2.0 ** -9)
    w["T"] = 2.0 ** -5
    choice = autotune(w, "fp64", steps=2)
    _say(f"fp64 autotune choice {choice}")
    ref = oracle.run(w)[0]
    with _ssm(w, "fp64", targets_per_lane=choice["targets_per_lane"],
              sources_per_item=choice["sources_per_item"], pair_scheme=choice["pair_scheme"]) as s:
        assert s.info()["pair_scheme"] == choice["pair_scheme"]
        s.run()
        assert _err(s.state(0), ref) <= FP64_TOL


def test_profile_stride_times_the_sampled_ticks_only(torch_cuda):
    """ssm_profile(every = k): events around the launches of ticks with
    tick % k == 0; every = 0 switches timing off; the run itself is unchanged."""
    from paper_2105_09688_amd import SSMError
    w = W.small_parity(n_ens=1, N=700)
    # both on the multi-launch path (a profiling context runs it)
    with _ssm(w, "fp32_kahan", persistent=-1) as a, _ssm(w, "fp32_kahan", persistent=-1) as b:
        a.profile(True, every=4)
        a.step(16)
        b.step(16)
        ia = a.info()
        assert ia["pair_launches"] == 4 and ia["update_launches"] == 4
        assert ia["pair_ms"] > 0.0
        assert np.array_equal(a.state(0), b.state(0))
        a.profile(False)
        a.step(4)
        assert a.info()["pair_launches"] == 0
        with pytest.raises(SSMError):
            a.profile(True, every=-1)
