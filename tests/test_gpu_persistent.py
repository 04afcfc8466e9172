"""Persistent runs of small systems (ssm_config.persistent): every tick of an
ssm_step call in one cooperative launch, one workgroup per 64 particles, one
barrier per system and tick.

The scheme is the same step (2.3)-(2.4) as the multi-launch path; only the
summation order differs (every ordered pair of the interaction in eq. (2.4)
in place of each unordered pair once, and tile sums for the measures' means),
so both are held to the oracle at the same pathwise bars (FP64 1e-10, FP32
1e-4) and to each other at rounding level.  The Brownian increments are the
same stream sums, bit for bit.
"""
import os
import sys

import numpy as np
import pytest

import oracle
from paper_2105_09688_amd import workloads as W

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10
FP32_TOL = 1e-4
TOL = {"fp64": FP64_TOL, "fp32": FP32_TOL, "fp32_kahan": FP32_TOL}


def _say(msg):
    print(f"[gpu-persistent] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    return torch


def _ssm(w, precision, **kw):
    from paper_2105_09688_amd.ssm import SSM
    return SSM(w, precision=precision, **kw)


def _err(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.max(np.abs(got - ref) / np.maximum(1.0, np.abs(ref)))) if ref.size else 0.0


def _run(w, precision, steps=None, **kw):
    with _ssm(w, precision, **kw) as s:
        if steps is None:
            s.run()
        else:
            for n in steps:
                s.step(n)
            s.sync()
        return s.states(), s.info()


@pytest.fixture(scope="module")
def small_case():
    """The small parity case: 10 ensembles x N = 1000, d = 1, h = 2^-8, 256 steps."""
    w = W.small_parity()
    return w, oracle.run(w)


@pytest.mark.parametrize("precision", ["fp64", "fp32_kahan", "fp32"])
def test_small_case_persistent_matches_oracle_and_multi_launch(torch_cuda, small_case, precision):
    """The whole small case in one launch (the library default there) against
    the oracle, and against the multi-launch path (persistent = -1)."""
    w, ref = small_case
    got, info = _run(w, precision)
    assert info["persistent"] == 1 and info["persistent_tiles"] == 160
    assert info["persistent_launches"] == 1 and info["persistent_ticks"] == 256
    assert info["newton_failures"] == 0 and info["nonfinite"] == 0 and info["newton_max_seen"] > 0
    multi, minfo = _run(w, precision, persistent=-1)
    assert minfo["persistent"] == 0 and minfo["persistent_launches"] == 0
    e_or = max(_err(g, r) for g, r in zip(got, ref))
    e_ml = max(_err(g, m) for g, m in zip(got, multi))
    _say(f"small case {precision}: persistent vs oracle {e_or:.3e}, vs multi-launch {e_ml:.3e}")
    assert e_or <= TOL[precision]
    assert e_ml <= (1e-13 if precision == "fp64" else 1e-5)


def _ragged(d):
    base = {1: W.small_parity(n_ens=1, N=8, h=2.0 ** -6, h_fine=2.0 ** -8),
            2: W.surrogate_d2(N=8, h=2.0 ** -6, h_fine=2.0 ** -8),
            3: W.precision_d3(N=8, h=2.0 ** -6)}
    if d == 4:
        w = W.precision_d3(N=8, h=2.0 ** -6)
        w.update(d=4, x0_mean=[0.2, -0.1, 0.0, 0.3], x0_std=[0.8, 1.0, 0.6, 0.9],
                 sigma=dict(s0=[0.2, 0.25, 0.15, 0.3], s1=[0.1, 0.0, 0.05, 0.1], s2=[0.0, 0.1, 0.0, 0.0]))
        w["b"]["ell"] = 0.7
    else:
        w = base[d]
    # one particle, one partial tile, exactly one tile, a tile and one, several tiles
    w = W.with_systems(w, [(1, 0, 2.0 ** -6), (63, 1, 2.0 ** -6), (64, 2, 2.0 ** -6), (65, 3, 2.0 ** -6),
                           (257, 4, 2.0 ** -6), (1000, 5, 2.0 ** -6)])
    w["T"] = 8 * 2.0 ** -6
    return w


@pytest.mark.parametrize("d", [1, 2, 3, 4])
@pytest.mark.parametrize("precision", ["fp64", "fp32_kahan"])
def test_ragged_sizes_and_dimensions(torch_cuda, d, precision):
    """Systems of 1, 63, 64, 65, 257 and 1000 particles in one context (tiles
    of 64: partial, exact, one over), d = 1..4, against the oracle."""
    w = _ragged(d)
    ref = oracle.run(w)
    got, info = _run(w, precision, persistent=1)
    assert info["persistent_tiles"] == 1 + 1 + 1 + 2 + 5 + 16
    errs = [_err(g, r) for g, r in zip(got, ref)]
    _say(f"ragged d={d} {precision}: per-system errors {['%.2e' % e for e in errs]}")
    assert max(errs) <= TOL[precision]


@pytest.mark.parametrize("family", ["gl_v2", "poly", "cucker_smale"])
@pytest.mark.parametrize("precision", ["fp64", "fp32_kahan"])
def test_paper_families_persistent(torch_cuda, family, precision):
    """The paper's families at one step size: Ginzburg-Landau version 2 (v
    sees mean(mu^X): two barriers per tick), the polynomial drift (v sees
    the second moment of mu^X) and Cucker-Smale (component-wise cubic, the
    linear extension of b, d = 2), against the oracle."""
    w = {"gl_v2": lambda: W.ginzburg_landau(version=2, n_ens=3, N=600, h=2.0 ** -6, h_fine=2.0 ** -8),
         "poly": lambda: W.polynomial_drift(n_ens=3, N=600, h=2.0 ** -6, h_fine=2.0 ** -8),
         "cucker_smale": lambda: W.cucker_smale(n_ens=3, N=600, h=2.0 ** -6, h_fine=2.0 ** -8)}[family]()
    w["T"] = 0.25
    ref = oracle.run(w)
    got, info = _run(w, precision, persistent=1)
    assert info["persistent_ticks"] == 16
    err = max(_err(g, r) for g, r in zip(got, ref))
    _say(f"{family} {precision}: {err:.3e}")
    assert err <= TOL[precision]


@pytest.mark.parametrize("family", ["small", "poly"])
@pytest.mark.parametrize("precision", ["fp64", "fp32_kahan"])
def test_split_launches_are_bitwise_one_launch(torch_cuda, family, precision):
    """A run in one ssm_step, in steps of 1 and in uneven pieces: the same
    final states bit for bit (each launch starts from the saved X and Y*;
    with a measure-dependent v the first Y* is solved again at the tile
    sums' moments, as inside a launch)."""
    w = (W.small_parity(n_ens=3, N=700, h=2.0 ** -6, h_fine=2.0 ** -8) if family == "small"
         else W.polynomial_drift(n_ens=3, N=700, h=2.0 ** -6, h_fine=2.0 ** -8))
    w["T"] = 0.25
    one, _ = _run(w, precision, persistent=1)
    ones, info = _run(w, precision, steps=[1] * 16, persistent=1)
    assert info["persistent_launches"] == 16
    pieces, _ = _run(w, precision, steps=[3, 1, 7, 5], persistent=1)
    for a, b, c in zip(one, ones, pieces):
        assert np.array_equal(a, b) and np.array_equal(a, c)


@pytest.mark.parametrize("precision", ["fp64", "fp32_kahan"])
def test_several_step_sizes(torch_cuda, precision):
    """A batch of ensembles of uneven N at three step sizes on one fine grid
    (strides 1, 2, 4) and the polynomial family at three levels: each system
    steps on its own ticks and draws its increments directly; against the
    oracle, and against the multi-launch path (shared Brownian windows,
    another association of the same sums)."""
    cases = [W.batched(n_ens=3, levels=(5, 6, 7), h_fine=2.0 ** -9, sizes=[300, 1000, 65]),
             W.polynomial_drift(n_ens=2, N=400, h_fine=2.0 ** -9, levels=(5, 6, 7))]
    for w in cases:
        w["T"] = 0.25
        ref = oracle.run(w)
        got, info = _run(w, precision, persistent=1)
        assert info["persistent_ticks"] == 32
        multi, _ = _run(w, precision, persistent=-1)
        e_or = max(_err(g, r) for g, r in zip(got, ref))
        e_ml = max(_err(g, m) for g, m in zip(got, multi))
        _say(f"several h {precision}: vs oracle {e_or:.3e}, vs multi-launch {e_ml:.3e}")
        assert e_or <= TOL[precision]
        assert e_ml <= (1e-13 if precision == "fp64" else 1e-5)


def test_switch_to_multi_launch_inside_a_window(torch_cuda):
    """Strides 1, 2, 4 with shared windows: persistent ticks end in the middle
    of a window, profiled (multi-launch) ticks continue (the window of the
    current period is drawn first), then persistent ticks again."""
    w = W.batched(n_ens=2, levels=(5, 6, 7), h_fine=2.0 ** -9, sizes=[300, 129])
    w["T"] = 0.25
    ref = oracle.run(w)
    with _ssm(w, "fp64", persistent=1) as s:
        s.step(5)
        s.profile(True, every=1)
        s.step(6)
        s.profile(False)
        s.run()
        got = s.states()
        info = s.info()
    assert info["persistent_launches"] == 2 and info["persistent_ticks"] == 26
    err = max(_err(g, r) for g, r in zip(got, ref))
    _say(f"window switch: {err:.3e}")
    assert err <= FP64_TOL


def test_long_calls_are_split_into_launches(torch_cuda):
    """A call of 8192 ticks runs as two launches of at most 4096 ticks (so
    that one call does not hold the GPU for an unbounded time), against the
    oracle."""
    w = W.small_parity(n_ens=2, N=100, h=2.0 ** -13, h_fine=2.0 ** -13)
    ref = oracle.run(w)
    got, info = _run(w, "fp64", persistent=1)
    assert info["persistent_ticks"] == 8192 and info["persistent_launches"] == 2
    err = max(_err(g, r) for g, r in zip(got, ref))
    _say(f"8192 ticks in two launches: {err:.3e}")
    assert err <= FP64_TOL


def test_mixed_with_multi_launch_ticks(torch_cuda, small_case):
    """Persistent ticks, then profiled ticks (the multi-launch path, whose
    block sums of Y* are refreshed first), then persistent ticks again: the
    run still matches the oracle."""
    w, ref = small_case
    with _ssm(w, "fp64") as s:
        s.step(40)
        s.profile(True, every=1)
        s.step(30)
        assert s.info()["pair_launches"] == 30
        s.profile(False)
        s.run()
        info = s.info()
        got = s.states()
    assert info["persistent_launches"] == 2 and info["persistent_ticks"] == 226
    err = max(_err(g, r) for g, r in zip(got, ref))
    _say(f"mixed: {err:.3e}")
    assert err <= FP64_TOL


def test_brownian_increments_bitwise_as_multi_launch(torch_cuda):
    """Pure noise, b = 0 and constant sigma: X_T = X_0 + sigma (sum of the
    increments), so both paths give the same states bit for bit exactly when
    they draw the same increments."""
    w = W.small_parity(n_ens=2, N=300, h=2.0 ** -5, h_fine=2.0 ** -9)
    w["T"] = 0.25
    w["v"] = dict(rho=0.0, a=0.0, kappa=0.0, lam=0.0)
    w["b"] = dict(c0=0.0, lam=0.0, g=0.0, ell=1.0)
    w["sigma"] = dict(s0=[0.7], s1=[0.0], s2=[0.0])
    for precision in ("fp64", "fp32_kahan"):
        a, ia = _run(w, precision, persistent=1)
        b, ib = _run(w, precision, persistent=-1)
        assert ia["persistent_ticks"] == 8 and ib["persistent_ticks"] == 0
        for x, y in zip(a, b):
            assert np.array_equal(x, y), precision


def test_required_mode_is_refused_where_ineligible(torch_cuda):
    """persistent = 1 fails at init for a system whose positions exceed the
    LDS budget and for the per-pair compensated study variant; persistent = 0
    then falls back."""
    from paper_2105_09688_amd import SSMError
    with pytest.raises(SSMError, match="kahan_span"):
        _ssm(W.small_parity(n_ens=1, N=300), "fp32_kahan", persistent=1, kahan_span=1)
    big = W.small_parity(n_ens=1, N=8192, h=2.0 ** -6, h_fine=2.0 ** -8)
    with pytest.raises(SSMError, match="KiB"):
        _ssm(big, "fp64", persistent=1)
    with _ssm(big, "fp64") as s:
        assert s.info()["persistent"] == 0
    with _ssm(W.small_parity(n_ens=1, N=300), "fp64", targets_per_lane=1) as s:
        assert s.info()["persistent"] == 0  # an explicit pair tiling keeps the multi-launch path


def test_default_choice_and_a_full_lds_system(torch_cuda):
    """One system of N = 8192 (d = 1, FP32-compensated): its positions fill
    the 32 KiB of LDS and it takes 128 tiles.  The default keeps it on the
    multi-launch path (the estimate: 28.6 us persistent against 19.9 us, the
    ordered pairs of a tile on one compute unit against the symmetric pairs
    over the chip); persistent = 1 runs it, against the oracle.  The small
    case takes the persistent path by default."""
    w = W.small_parity(n_ens=1, N=8192, h=2.0 ** -6, h_fine=2.0 ** -8)
    w["T"] = 4 * 2.0 ** -6
    with _ssm(w, "fp32_kahan") as s:
        assert s.info()["persistent"] == 0
    ref = oracle.run(w)
    got, info = _run(w, "fp32_kahan", persistent=1)
    assert info["persistent_tiles"] == 128 and info["persistent_ticks"] == 4
    err = _err(got[0], ref[0])
    _say(f"N=8192 persistent: {err:.3e}")
    assert err <= FP32_TOL
    with _ssm(W.small_parity(), "fp64") as s:
        assert s.info()["persistent"] == 1


def test_barrier_timeout_aborts_cleanly(torch_cuda):
    """A barrier wait limit of zero, set from the host for one context
    (SSM_PERSISTENT_WAIT_US=0 at ssm_init): the first wait that is not
    already satisfied runs out, every workgroup leaves at its next barrier,
    ssm_sync reports the abort and the context refuses further steps, while a
    context created afterwards runs normally.  (Every kernel exits normally;
    the GPU is not left waiting.)"""
    from paper_2105_09688_amd import SSMError
    # v depends on mu^X: the barrier between the update and the implicit step
    # has no work between arriving and waiting, so its first arriver waits
    w = W.polynomial_drift(n_ens=2, N=1000)
    os.environ["SSM_PERSISTENT_WAIT_US"] = "0"
    try:
        s = _ssm(w, "fp64", persistent=1)
    finally:
        del os.environ["SSM_PERSISTENT_WAIT_US"]
    with s:
        s.step(64)
        with pytest.raises(SSMError, match="barrier"):
            s.sync()
        _say("abort reported")
        with pytest.raises(SSMError, match="aborted"):
            s.step(1)
    ref = oracle.run(W.with_systems(w, [(1000, 0, w["systems"][0][2])]), stop_after=8)[0]
    with _ssm(w, "fp64", persistent=1) as ok:
        ok.step(8)
        ok.sync()
        assert _err(ok.state(0), ref) <= FP64_TOL
