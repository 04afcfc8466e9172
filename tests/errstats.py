"""Error statistics of Section 3 in plain numpy, applied to GPU results in the
tests (the oracle's own functions only ever see oracle data).

strong_error: epsilon_2 = ((1/N) sum_j |X^j - X_ref^j|^2)^(1/2) over the
    particles of all listed systems;
weak_error:   epsilon_1 = |(1/N) sum_j (X^j - X_ref^j)|_2;
ols_slope:    least-squares slope of log2(err) against log2(h).
"""
import numpy as np


def _pairs(X, X_ref):
    if isinstance(X, (list, tuple)):
        return [(np.atleast_2d(np.asarray(a, dtype=np.float64)), np.atleast_2d(np.asarray(b, dtype=np.float64)))
                for a, b in zip(X, X_ref)]
    return [(np.atleast_2d(np.asarray(X, dtype=np.float64)), np.atleast_2d(np.asarray(X_ref, dtype=np.float64)))]


def strong_error(X, X_ref) -> float:
    ps = _pairs(X, X_ref)
    num = sum(float(np.sum((a - b) ** 2)) for a, b in ps)
    return float(np.sqrt(num / sum(a.shape[1] for a, _ in ps)))


def weak_error(X, X_ref) -> float:
    D = np.concatenate([a - b for a, b in _pairs(X, X_ref)], axis=1)
    return float(np.linalg.norm(D.mean(axis=1)))


def ols_slope(hs, errs) -> float:
    return float(np.polyfit(np.log2(np.asarray(hs, dtype=np.float64)), np.log2(np.asarray(errs, dtype=np.float64)), 1)[0])
