"""The tests' numpy error statistics (used on GPU results) and the oracle's
(used on oracle results) are two writings of the same definitions of
Section 3: they agree on random data, and on cases with known values."""
import numpy as np

import errstats
import oracle


def test_errstats_agree_with_the_oracle():
    rng = np.random.default_rng(0)
    X = [rng.normal(size=(2, n)) for n in (5, 17, 1)]
    R = [x + rng.normal(size=x.shape) * 0.1 for x in X]
    assert abs(errstats.strong_error(X, R) - oracle.strong_error(X, R)) <= 1e-15
    assert abs(errstats.weak_error(X, R) - oracle.weak_error(X, R)) <= 1e-15
    hs, es = [2.0 ** -k for k in range(4, 9)], [0.3 * (2.0 ** -k) ** 0.5 * (1 + 0.01 * k) for k in range(4, 9)]
    assert abs(errstats.ols_slope(hs, es) - oracle.ols_slope(hs, es)) <= 1e-12


def test_errstats_known_values():
    X = [np.array([[1.0, 2.0, 3.0]]), np.array([[0.0]])]
    R = [np.array([[0.0, 2.0, 1.0]]), np.array([[1.0]])]
    # differences 1, 0, 2, -1: mean square 6/4, mean 2/4
    assert abs(errstats.strong_error(X, R) - np.sqrt(1.5)) <= 1e-15
    assert abs(errstats.weak_error(X, R) - 0.5) <= 1e-15
    assert abs(errstats.ols_slope([0.25, 0.5, 1.0], [1.0, 2.0, 4.0]) - 1.0) <= 1e-12
