"""Checkpoint and resume through the C ABI, non-finite particles, and the
surrogate's fallback after the state or the weights change.

A run stopped after n steps and continued in a fresh context from the state
and step count that ssm_get_state returned (ssm_set_state with the step)
must equal the uninterrupted run bitwise: the step n + 1 of (2.3)-(2.4)
draws the increment dW_n of the same Brownian path (Section 3 compares step
sizes on the same paths), and every reduction runs in a fixed order.
"""
import sys

import numpy as np
import pytest

from paper_2105_09688_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-resume] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    return torch


def _ssm(w, precision, **kw):
    from paper_2105_09688_amd.ssm import SSM
    return SSM(w, precision=precision, **kw)


def _small():
    w = W.small_parity(n_ens=3, N=700, h=2.0 ** -6, h_fine=2.0 ** -8)
    w["T"] = 0.25
    return w


def _poly():
    # v depends on mu^X (second moment): the unfused path
    w = W.polynomial_drift(n_ens=2, N=513, h=2.0 ** -6, h_fine=2.0 ** -8)
    w["T"] = 0.25
    return w


def _batched():
    # two step sizes in one context (strides 1 and 2): resume at an even tick
    w = W.batched(n_ens=2, levels=(6, 7), h_fine=2.0 ** -9, sizes=[300, 129])
    w["T"] = 0.25
    return w


CASES = {"small_fused": _small, "poly_unfused": _poly, "batched_two_h": _batched}


@pytest.mark.parametrize("precision", ["fp64", "fp32_kahan"])
@pytest.mark.parametrize("case", sorted(CASES))
def test_resume_in_fresh_context_is_bitwise(torch_cuda, case, precision):
    """Run to T; run to tick t, save every system with its step count,
    destroy the context, restore into a fresh one and run to T: the two final
    states (and Y*) are equal bitwise."""
    w = CASES[case]()
    _say(f"resume {case} {precision}")
    with _ssm(w, precision) as a:
        a.run()
        want = [a.state(s) for s in range(len(a.N))]
        total = a.info()["ticks_total"]
    t = total // 2
    if t % 2:
        t -= 1
    saved = []
    with _ssm(w, precision) as b:
        b.step(t)
        for s in range(len(b.N)):
            X, n = b.state_step(s)
            saved.append((X, n))
    with _ssm(w, precision) as c:
        for s, (X, n) in enumerate(saved):
            c.set_state(s, X, step=n)
        assert c.info()["tick"] == t
        c.run()
        got = [c.state(s) for s in range(len(c.N))]
    for s, (g, r) in enumerate(zip(got, want)):
        assert np.array_equal(g, r), (case, precision, s, float(np.max(np.abs(g - r))))


def test_set_state_step_is_validated(torch_cuda):
    """Systems (300, h = 2^-6), (300, 2^-7), (129, 2^-6), (129, 2^-7): a tick
    is 2^-7 and every system steps on even ticks.  A step of system 1 (one
    tick per step) at an odd tick, one past T and a negative one other than
    -1 are refused; -1 keeps the tick; step 2 of system 0 (two ticks per
    step) is tick 4."""
    from paper_2105_09688_amd import SSMError
    w = _batched()
    with _ssm(w, "fp64") as c:
        X1 = c.state(1)
        for bad in (1, 3, 10 ** 6, -2):
            with pytest.raises(SSMError) as e:
                c.set_state(1, X1, step=bad)
            assert e.value.status == -1, bad
        c.step(2)
        c.set_state(1, X1, step=-1)
        assert c.info()["tick"] == 2
        c.set_state(0, c.state(0), step=2)
        assert c.info()["tick"] == 4
        assert c.state_step(1)[1] == 4 and c.state_step(0)[1] == 2


@pytest.mark.parametrize("precision", ["fp64", "fp32_kahan"])
def test_nonfinite_particle_is_reported(torch_cuda, precision):
    """A state with one NaN particle, written through ssm_set_state (a
    corrupted particle forced from the host): the implicit solve that follows
    flags it, ssm_sync reports SSM_ERR_NONFINITE (-3) from then on, the
    counter is positive, and every kernel still finishes (the NaN spreads
    through the pair sums, as it would in a real blow-up)."""
    from paper_2105_09688_amd import SSMError
    w = W.small_parity(n_ens=1, N=1000, h=2.0 ** -6, h_fine=2.0 ** -6)
    w["T"] = 0.25
    with _ssm(w, precision) as s:
        s.step(2)
        s.sync()
        assert s.info()["nonfinite"] == 0
        X = s.state(0)
        X[0, 123] = np.nan
        _say(f"nonfinite {precision}: set_state with a NaN particle")
        with pytest.raises(SSMError) as e:
            s.set_state(0, X)
        assert e.value.status == -3
        s.step(1)
        with pytest.raises(SSMError) as e:
            s.sync()
        assert e.value.status == -3
        info = s.info()
        assert info["nonfinite"] > 0 and info["newton_failures"] == 0
        _say(f"nonfinite count {info['nonfinite']}")
    # an infinite coordinate is flagged the same way, and a clean context is not affected
    with _ssm(w, precision) as s, _ssm(w, precision) as clean:
        X = s.state(0)
        X[0, 7] = np.inf
        with pytest.raises(SSMError) as e:
            s.set_state(0, X)
        assert e.value.status == -3
        clean.step(3)
        clean.sync()
        assert clean.info()["nonfinite"] == 0


def test_surrogate_falls_back_after_set_state_and_reload(torch_cuda):
    """Residuals and gains belong to the state and the weights of their
    check: after ssm_set_state (or a weight reload) the ticks up to the next
    check use the exact pair sums (no surrogate tick is counted), and the
    surrogate resumes after that check."""
    from paper_2105_09688_amd.ssm import mlp_num_params
    w = W.surrogate_d2(N=1024, h=2.0 ** -9, h_fine=2.0 ** -9)
    w["T"] = 32 * 2.0 ** -9
    zeros = np.zeros(mlp_num_params(2), dtype=np.float32)
    with _ssm(w, "fp32_kahan") as s:
        s.surrogate_load(zeros)
        s.surrogate_enable(check_every=4, tol=1e9, mode="residual")
        s.step(7)  # checks at ticks 0, 4; network at 1-3, 5-6
        i0 = s.info()
        assert i0["surr_checks"] == 2 and i0["surr_ticks"] == 5 and i0["surr_fallback_ticks"] == 0
        s.set_state(0, s.state(0))
        s.step(1)  # tick 7: exact
        i1 = s.info()
        assert i1["surr_ticks"] == 5 and i1["surr_fallback_ticks"] == 1
        s.step(2)  # tick 8: check (passes), tick 9: network
        i2 = s.info()
        assert i2["surr_checks"] == 3 and i2["surr_ticks"] == 6
        s.step(2)  # ticks 10, 11: network
        s.surrogate_load(zeros)
        s.step(1)  # tick 12 is a check anyway
        s.step(1)  # tick 13: network again after the check
        i3 = s.info()
        assert i3["surr_ticks"] == 9 and i3["surr_checks"] == 4
        s.step(1)  # tick 14
        s.surrogate_load(zeros)
        s.step(1)  # tick 15: exact (reloaded weights, no check since)
        i4 = s.info()
        assert i4["surr_ticks"] == 10 and i4["surr_fallback_ticks"] == 2
