"""The mean-square stability constant beta of Theorem 2.9 as bench.py
evaluates it, against what the paper states about it (no GPU)."""
import math

import numpy as np
import pytest

import bench


def test_ou_condition_of_section_3_4_1():
    """OU (Section 3.4.1): L_v = rho, L_bt = lam^2, the other constants 0; the
    paper derives beta < 0 exactly when h < -(2 rho + 2 lam + 1) / lam^2
    (lam > 0, rho + lam < -1/2)."""
    for rho, lam in ((-2.0, 0.5), (-1.5, 0.9), (-3.0, 2.0)):
        h_star = -(2 * rho + 2 * lam + 1) / lam ** 2
        for f in (0.5, 0.9, 0.99):
            h = f * h_star
            if 1 - h * (2 * rho + 1) <= 0:
                continue
            assert bench.stability_beta(h, L_v=rho, L_b=0.0, L_bt=lam ** 2, L_s=0.0) < 0
        for f in (1.01, 1.1, 2.0):
            h = f * h_star
            if 1 - h * (2 * rho + 1) <= 0:
                continue
            assert bench.stability_beta(h, L_v=rho, L_b=0.0, L_bt=lam ** 2, L_s=0.0) > 0


def test_one_plus_beta_h_is_positive_under_the_step_condition():
    """Theorem 2.9: under the step condition of Theorem 2.6 (1 - h(2 L_v + 1) > 0)
    the factor 1 + beta h is always positive."""
    rng = np.random.default_rng(3)
    for _ in range(2000):
        L_v = rng.normal() * 3
        L_b, L_bt, L_s, L_st, L_vt = np.abs(rng.normal(size=5)) * 2
        hmax = 1.0 / (2 * L_v + 1) if 2 * L_v + 1 > 0 else 10.0
        h = rng.uniform(0, 1) * hmax
        if not (1 - h * (2 * L_v + 1) > 0):
            continue
        assert 1 + bench.stability_beta(h, L_v, L_b, L_bt, L_s, L_st, L_vt) * h > 0


def test_beta_is_undefined_outside_the_step_condition():
    with pytest.raises(ValueError):
        bench.stability_beta(0.1, L_v=4.5, L_b=0.0, L_bt=1.0, L_s=1.0)  # 1 - h (2 L_v + 1) = 0
    with pytest.raises(ValueError):
        bench.gl_stability_beta(-12.0, 0.1)


def test_section_3_4_2_statements():
    """Section 3.4.2 (L_v = -5/2 - gamma, L_bt = L_s = 1, L_b = gamma^2): with
    gamma = 0 only a small h gives beta < 0; at h = 0.1 the factor 1 + beta h
    exceeds 1 for gamma >= 5 (loss of the guarantee); sufficient condition of
    Theorem 2.9: L_v < -(1 + A)/2 gives beta < 0 for small h."""
    assert bench.gl_stability_beta(0.0, 1e-2) < 0
    assert bench.gl_stability_beta(0.0, 1e-4) < 0
    assert bench.gl_stability_beta(0.0, 2.0) > 0
    for g in range(5, 13):
        assert 1 + bench.gl_stability_beta(float(g), 0.1) * 0.1 > 1
    # the sufficient condition, and the h -> 0 limit beta -> 2 L_v + A + 1
    for g in (-0.2, 0.0, 0.2):
        A = 2 * abs(g) + 2 + 1
        L_v = -2.5 - g
        assert L_v < -(1 + A) / 2
        assert bench.gl_stability_beta(g, 1e-9) == pytest.approx(2 * L_v + A + 1, rel=1e-6)
        assert bench.gl_stability_beta(g, 1e-3) < 0


def test_study_error_helpers_match_the_oracle_definitions(oracle_mod):
    """The studies compute strong and weak errors and slopes with their own
    numpy helpers (a study may not call the oracle); they agree with the
    oracle's definitions (Section 3) on random lists of systems."""
    rng = np.random.default_rng(9)
    X = [rng.normal(size=(2, n)) for n in (5, 17, 64)]
    Y = [x + 0.1 * rng.normal(size=x.shape) + 0.01 for x in X]
    assert bench._rmse(X, Y) == pytest.approx(oracle_mod.strong_error(X, Y), rel=1e-12)
    assert bench._weak(X, Y) == pytest.approx(oracle_mod.weak_error(X, Y), rel=1e-12)
    hs = [2.0 ** -l for l in range(4, 9)]
    errs = [0.3 * h ** 0.5 * (1 + 0.05 * math.sin(l)) for l, h in enumerate(hs)]
    assert bench._slope(hs, errs) == pytest.approx(oracle_mod.ols_slope(hs, errs), rel=1e-10)

