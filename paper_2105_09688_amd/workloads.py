"""Seeded synthetic workloads for the SSM particle step.

This module holds inputs only: coefficient sets, sizes and seeded random
arrays.  It contains none of the scheme's arithmetic, imports neither the HIP
library nor the oracle, and is what both of them are fed from.

A workload is a plain dict (see ``oracle/__init__.py`` and
``paper_2105_09688_amd/ssm.py`` for the two consumers):

    d, systems=[(N, ens, h), ...], T, h_fine, seed,
    v={rho, a, kappa, lam}, b={c0, lam, g, ell}, sigma={s0, s1, s2},
    x0_mean, x0_std

Coefficient family (all examples of Section 3 except FitzHugh-Nagumo fit it):
    v(y, mu_X) = (rho - kappa m2(mu_X)) y - a |y|^2 y + lam mean(mu_X)
    b(y, mu_Y) = c0 y + lam mean(mu_Y) + g int (z - y) exp(-|y - z|^2 / (2 ell^2)) mu_Y(dz)
    sigma      = diag(s0 + s1 y + s2 mean(mu_Y))
"""
from __future__ import annotations

import copy

import numpy as np

# The d = 1 coefficients shared by the small parity case, the single-GPU
# throughput case and the batched case: cubic v of the Ginzburg-Landau family
# (Section 3.1), an odd Gaussian interaction in b and an affine sigma that
# depends on the mean of mu_Y.
_GAUSS_1D = dict(
    d=1,
    T=1.0,
    seed=0,
    v=dict(rho=0.0, a=1.0, kappa=0.0, lam=0.0),
    b=dict(c0=1.0, lam=0.0, g=1.0, ell=1.0),
    sigma=dict(s0=[0.0], s1=[0.3], s2=[0.2]),
    x0_mean=[1.0],
    x0_std=[0.5],
)


def small_parity(n_ens: int = 10, N: int = 1000, h: float = 2.0 ** -8, h_fine: float = 2.0 ** -12) -> dict:
    """d=1, N=1000 particles, 10 independent ensembles, T=1, h=2^-8 (256 steps), FP64.

    Brownian increments are sums over a 2^-12 grid so that a 2^-12 run is the
    proxy "true" solution on the same paths (Section 3).
    """
    w = copy.deepcopy(_GAUSS_1D)
    w["h_fine"] = h_fine
    w["systems"] = [(N, e, h) for e in range(n_ens)]
    return w


def single_gpu_d1(N: int = 2 ** 16, h: float = 2.0 ** -10, h_fine: float = 2.0 ** -14) -> dict:
    """d=1, N=2^16, T=1, h=2^-10 (1024 steps); fine Brownian grid 2^-14."""
    w = copy.deepcopy(_GAUSS_1D)
    w["h_fine"] = h_fine
    w["systems"] = [(N, 0, h)]
    return w


def precision_d3(N: int = 2 ** 18, h: float = 2.0 ** -10) -> dict:
    """d=3 precision study: radial cubic v, Gaussian interaction of width 0.5,
    diagonal sigma_k = 0.2 + 0.1 y_k, X0 ~ N(0, I), N=2^18, T=1, h=2^-10."""
    return dict(
        d=3, T=1.0, seed=0, h_fine=h,
        systems=[(N, 0, h)],
        v=dict(rho=0.0, a=1.0, kappa=0.0, lam=0.0),
        b=dict(c0=0.0, lam=0.0, g=1.0, ell=0.5),
        sigma=dict(s0=[0.2] * 3, s1=[0.1] * 3, s2=[0.0] * 3),
        x0_mean=[0.0] * 3, x0_std=[1.0] * 3,
    )


def batched_sizes(n_ens: int = 64, lo_log2: int = 10, hi_log2: int = 16, seed: int = 0) -> list:
    """Ensemble sizes log-uniform in [2^lo, 2^hi], seeded."""
    rng = np.random.Generator(np.random.Philox(key=seed + 2))
    u = rng.random(n_ens)
    N = np.clip(np.rint(2.0 ** (lo_log2 + (hi_log2 - lo_log2) * u)), 2 ** lo_log2, 2 ** hi_log2)
    return [int(n) for n in N]


def batched(n_ens: int = 64, levels=(4, 5, 6, 7, 8), h_fine: float = 2.0 ** -12, sizes=None) -> dict:
    """d=1 batched case: ensembles of uneven N, several step sizes 2^-l on one
    fine Brownian grid, T=1.  One system per (ensemble, level)."""
    w = copy.deepcopy(_GAUSS_1D)
    w["h_fine"] = h_fine
    sizes = batched_sizes(n_ens) if sizes is None else list(sizes)
    w["systems"] = [(N, e, 2.0 ** -l) for e, N in enumerate(sizes) for l in levels]
    return w


def surrogate_d2(N: int = 2 ** 20, h: float = 2.0 ** -9, h_fine: float = 2.0 ** -13) -> dict:
    """d=2: radial cubic v, unit-width Gaussian interaction, sigma = 0.25 I + 0.1 diag(y),
    X0 ~ N(0, I), N=2^20, T=1, h=2^-9."""
    return dict(
        d=2, T=1.0, seed=0, h_fine=h_fine,
        systems=[(N, 0, h)],
        v=dict(rho=0.0, a=1.0, kappa=0.0, lam=0.0),
        b=dict(c0=0.0, lam=0.0, g=1.0, ell=1.0),
        sigma=dict(s0=[0.25] * 2, s1=[0.1] * 2, s2=[0.0] * 2),
        x0_mean=[0.0] * 2, x0_std=[1.0] * 2,
    )


def ou(rho: float = -1.0, lam: float = 0.5, eta: float = 0.3, x0: float = 1.0, x0_std: float = 0.0,
       N: int = 1000, h: float = 2.0 ** -6, n_ens: int = 1, T: float = 1.0, h_fine=None) -> dict:
    """Linear Ornstein-Uhlenbeck MV-SDE of Section 3.4.1: v = rho x, b = lam E[X], sigma = eta."""
    return dict(
        d=1, T=T, seed=0, h_fine=h if h_fine is None else h_fine,
        systems=[(N, e, h) for e in range(n_ens)],
        v=dict(rho=rho, a=0.0, kappa=0.0, lam=0.0),
        b=dict(c0=0.0, lam=lam, g=0.0, ell=1.0),
        sigma=dict(s0=[eta], s1=[0.0], s2=[0.0]),
        x0_mean=[x0], x0_std=[x0_std],
    )


def ginzburg_landau(version: int = 1, n_ens: int = 10, N: int = 1000, h: float = 2.0 ** -8,
                    h_fine: float = 2.0 ** -12, sigma_p: float = 1.5, c: float = 0.5, x0: float = 1.0,
                    levels=None) -> dict:
    """Stochastic Ginzburg-Landau MV-SDE of Section 3.1,
    dX = ((s'^2 / 2) X - X^3 + c E[X]) dt + s' X dW, X_0 = x0, with s' = 1.5,
    c = 0.5, x0 = 1, T = 1, N = 1000.  SSM version 1 puts c E[X] in b (at
    mu_Y), version 2 in v (at mu_X, the implicit step's measure).  With
    `levels`, one system per (ensemble, step 2^-l) on the fine grid."""
    if version not in (1, 2):
        raise ValueError("version is 1 or 2")
    systems = ([(N, e, h) for e in range(n_ens)] if levels is None
               else [(N, e, 2.0 ** -l) for e in range(n_ens) for l in levels])
    return dict(
        d=1, T=1.0, seed=0, h_fine=h_fine, systems=systems,
        v=dict(rho=0.0, a=1.0, kappa=0.0, lam=c if version == 2 else 0.0),
        b=dict(c0=sigma_p ** 2 / 2, lam=c if version == 1 else 0.0, g=0.0, ell=1.0),
        sigma=dict(s0=[0.0], s1=[sigma_p], s2=[0.0]),
        x0_mean=[x0], x0_std=[0.0],
    )


def polynomial_drift(gamma: float = -1.0, n_ens: int = 10, N: int = 1000, h: float = 2.0 ** -8,
                     h_fine: float = 2.0 ** -12, x0: float = 1.0, T: float = 1.0, levels=None) -> dict:
    """Polynomial-drift MV-SDE of Section 3.3,
    dX = (gamma X + E[X] - X E[|X|^2]) dt + X dW, with v = gamma x - x E|X|^2
    (at mu_X), b = E[X] (at mu_Y), sigma = x; gamma = -1, N = 1000.  The paper
    gives T = 1 and T = 2 in two places and no x0: T = 1 and x0 = 1 here."""
    systems = ([(N, e, h) for e in range(n_ens)] if levels is None
               else [(N, e, 2.0 ** -l) for e in range(n_ens) for l in levels])
    return dict(
        d=1, T=T, seed=0, h_fine=h_fine, systems=systems,
        v=dict(rho=gamma, a=0.0, kappa=1.0, lam=0.0),
        b=dict(c0=0.0, lam=1.0, g=0.0, ell=1.0),
        sigma=dict(s0=[0.0], s1=[1.0], s2=[0.0]),
        x0_mean=[x0], x0_std=[0.0],
    )


def cucker_smale(lam: float = 2.0, sigma_p: float = 4.0, n_ens: int = 10, N: int = 1000, h: float = 2.0 ** -8,
                 h_fine: float = 2.0 ** -12, T: float = 2.0, levels=None) -> dict:
    """Two-dimensional Cucker-Smale flocking model of Section 3.4.3, state
    (V, X): dV = (1 - V^3 + lam (mean V - V)) dt + sigma' (mean V - V) dW,
    dX = V dt, with lam = 2, sigma' = 4, T = 2, N = 1000.  Split as
    v = (-V^3, 0) (component-wise cubic), b = (1 + lam (mean V - V), V),
    sigma = (sigma' (mean V - V), 0).  The paper's coefficient line writes the
    mean terms as int (V - z) dmu(z) and its particle dynamics as
    (1/N) sum_j (V^j - V^i); the particle form (the one whose V converges to
    1, as the paper states) is used.  V_0 ~ N(1, 2) read as variance 2;
    X_0 = 0 (not given)."""
    systems = ([(N, e, h) for e in range(n_ens)] if levels is None
               else [(N, e, 2.0 ** -l) for e in range(n_ens) for l in levels])
    return dict(
        d=2, T=T, seed=0, h_fine=h_fine, systems=systems,
        v=dict(rho=0.0, a=0.0, kappa=0.0, lam=0.0, componentwise=True, a_k=[1.0, 0.0]),
        b=dict(c0=0.0, lam=0.0, g=0.0, ell=1.0, const=[1.0, 0.0], mat=[[-lam, 0.0], [1.0, 0.0]],
               mean=[lam, 0.0]),
        sigma=dict(s0=[0.0, 0.0], s1=[-sigma_p, 0.0], s2=[sigma_p, 0.0]),
        x0_mean=[1.0, 0.0], x0_std=[2.0 ** 0.5, 0.0],
    )


def gl_stability(gamma: float = 0.0, x0: float = 1.0, h: float = 1e-2, T: float = 3.0, N: int = 1000,
                 n_ens: int = 10, allow_unstable_h: bool = False) -> dict:
    """Stability example of Section 3.4.2: dX = (-5/2 X - 1/4 X^3 + E[X]) dt + X dW,
    X_0 = x0, split as v = -5/2 x - 1/4 x^3 - gamma x, b = E[X] + gamma x,
    sigma = x (gamma moves slope between v and b); N = 1000.  The Brownian
    increments are drawn at the step itself (h_fine = h).  allow_unstable_h
    lifts the step-size condition of Theorem 2.6 for steps the study takes on
    purpose (the implicit step stays uniquely solvable: 1 - h rho > 0)."""
    return dict(
        d=1, T=T, seed=0, h_fine=h, systems=[(N, e, h) for e in range(n_ens)],
        v=dict(rho=-2.5 - gamma, a=0.25, kappa=0.0, lam=0.0),
        b=dict(c0=gamma, lam=1.0, g=0.0, ell=1.0),
        sigma=dict(s0=[0.0], s1=[1.0], s2=[0.0]),
        x0_mean=[x0], x0_std=[0.0],
        allow_unstable_h=allow_unstable_h,
    )


def with_systems(w: dict, systems) -> dict:
    w = copy.deepcopy(w)
    w["systems"] = [tuple(s) for s in systems]
    return w


def with_h(w: dict, h: float) -> dict:
    """Same workload with every system stepping at h (same ensembles, same Brownian grid)."""
    w = copy.deepcopy(w)
    w["systems"] = [(N, e, h) for (N, e, _h) in w["systems"]]
    return w


def random_cloud(d: int, N: int, seed: int, loc: float = 0.0, scale: float = 1.0) -> np.ndarray:
    """A seeded Gaussian particle cloud, component-major [d][N], float64."""
    rng = np.random.Generator(np.random.Philox(key=seed + 1000))
    return loc + scale * rng.standard_normal((d, N))
