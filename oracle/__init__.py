"""FP64 CPU oracle of the split-step method (SSM), arXiv:2105.09688.

TEST INFRASTRUCTURE ONLY.  The test suite, the smoke check and the
CPU-baseline leg of the benchmark load this; the HIP library never does, and
this module imports nothing from it.  The arithmetic lives in
``ssm_oracle.c`` (plain C, double precision, ``-ffp-contract=off``); this file
marshals arguments and adds the error statistics of Section 3, which are plain
numpy expressions of their definitions.

A workload is a plain dict:

    {"d": 1, "systems": [(N, ens, h), ...], "T": 1.0, "h_fine": 2**-12,
     "seed": 0, "v": {"rho", "a", "kappa", "lam"}, "b": {"c0", "lam", "g", "ell"},
     "sigma": {"s0": [..], "s1": [..], "s2": [..]},
     "x0_mean": [..], "x0_std": [..]}

with the coefficient family documented in ``ssm_oracle.h``.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libssm_oracle.so")
_lib = None

MAX_D = 4
OK, ERR_INVALID, ERR_NEWTON, ERR_NONFINITE = 0, -1, -2, -3


class _Cfg(C.Structure):
    _fields_ = [
        ("d", C.c_int32), ("n_sys", C.c_int32),
        ("N", C.POINTER(C.c_int64)), ("ens", C.POINTER(C.c_int32)), ("h", C.POINTER(C.c_double)),
        ("T", C.c_double), ("h_fine", C.c_double), ("seed", C.c_uint64),
        ("v_rho", C.c_double), ("v_a", C.c_double), ("v_kappa", C.c_double), ("v_lam", C.c_double),
        ("b_c0", C.c_double), ("b_lam", C.c_double), ("b_g", C.c_double), ("b_ell", C.c_double),
        ("s0", C.c_double * MAX_D), ("s1", C.c_double * MAX_D), ("s2", C.c_double * MAX_D),
        ("x0_mean", C.c_double * MAX_D), ("x0_std", C.c_double * MAX_D),
        ("newton_max_iter", C.c_int32), ("allow_unstable_h", C.c_int32),
        ("v_componentwise", C.c_int32), ("pad", C.c_int32),
        ("v_ak", C.c_double * MAX_D), ("b_const", C.c_double * MAX_D), ("b_mat", C.c_double * (MAX_D * MAX_D)),
        ("b_mean", C.c_double * MAX_D),
    ]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b  # noqa: WPS433 -- compile on first use
        _b.build()
    lib = C.CDLL(_LIB_PATH)
    dp = C.POINTER(C.c_double)
    u64p = C.POINTER(C.c_uint64)
    lib.ssmo_philox4x64_10.argtypes = [u64p, u64p, u64p]
    lib.ssmo_normals4.argtypes = [C.c_uint64, C.c_uint32, C.c_uint64, C.c_uint64, C.c_uint64, dp]
    lib.ssmo_stream_normal.argtypes = [C.c_uint64, C.c_uint64, C.c_uint64, C.c_uint64]
    lib.ssmo_stream_normal.restype = C.c_double
    lib.ssmo_brownian.argtypes = [C.c_uint64, C.c_int, C.c_uint64, C.c_uint64, C.c_uint64, C.c_int64,
                                  C.c_double, dp]
    lib.ssmo_implicit.argtypes = [C.c_int, dp, C.c_double, C.c_double, C.c_double, C.c_double,
                                  C.c_double, dp, C.c_double, C.c_int, dp]
    lib.ssmo_implicit.restype = C.c_int
    lib.ssmo_drift.argtypes = [C.c_int, C.c_int64, dp, C.c_double, C.c_double, C.c_double,
                               C.c_double, dp]
    lib.ssmo_pair_sum.argtypes = [C.c_int, C.c_int64, dp, C.c_double, dp]
    lib.ssmo_pair_sum_at.argtypes = [C.c_int, C.c_int64, dp, C.c_double, C.c_int64,
                                     C.POINTER(C.c_int64), dp]
    lib.ssmo_step.argtypes = [C.POINTER(_Cfg), C.c_int32, C.c_int64, C.c_double, C.c_int64, dp, dp]
    lib.ssmo_step.restype = C.c_int
    lib.ssmo_step_at.argtypes = [C.POINTER(_Cfg), C.c_int32, C.c_int64, C.c_double, C.c_int64, dp, C.c_int64,
                                 C.POINTER(C.c_int64), dp]
    lib.ssmo_step_at.restype = C.c_int
    lib.ssmo_init_state.argtypes = [C.POINTER(_Cfg), C.c_int32, C.c_int64, dp]
    lib.ssmo_run.argtypes = [C.POINTER(_Cfg), C.c_int64, dp, C.POINTER(C.c_int64)]
    lib.ssmo_run.restype = C.c_int
    lib.ssmo_moments.argtypes = [C.c_int, C.c_int64, dp, dp, dp]
    lib.ssmo_rff_omegas.argtypes = [C.c_uint64, C.c_int, C.c_int, C.c_double, dp]
    lib.ssmo_rff_moments.argtypes = [C.c_int, C.c_int64, dp, C.c_int, dp, dp]
    lib.ssmo_mlp_num_params.argtypes = [C.c_int, C.c_int, C.c_int]
    lib.ssmo_mlp_num_params.restype = C.c_int64
    lib.ssmo_mlp_forward.argtypes = [C.c_int, C.c_int, C.c_int, dp, C.c_int64, dp, dp]
    lib.ssmo_mlp_loss_grad.argtypes = [C.c_int, C.c_int, C.c_int, dp, C.c_int64, dp, dp, dp]
    lib.ssmo_mlp_loss_grad.restype = C.c_double
    lib.ssmo_num_threads.restype = C.c_int
    lib.ssmo_set_num_threads.argtypes = [C.c_int]
    _lib = lib
    return lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


class OracleError(RuntimeError):
    pass


def _check(st: int, what: str):
    if st < 0:
        raise OracleError(f"{what}: oracle status {st}")


# ---------------------------------------------------------------- random numbers
def philox4x64_10(ctr, key) -> np.ndarray:
    """Philox4x64-10 block (Salmon et al., SC'11) of counter ``ctr`` under ``key``."""
    lib = _load()
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    u64p = C.POINTER(C.c_uint64)
    lib.ssmo_philox4x64_10(c.ctypes.data_as(u64p), k.ctypes.data_as(u64p), out.ctypes.data_as(u64p))
    return out


def normals4(seed: int, tag: int, i: int, n: int, e: int) -> np.ndarray:
    """Four standard normals of stream ``tag`` for particle ``i``, grid index ``n``, ensemble ``e``."""
    lib = _load()
    z = np.zeros(4)
    lib.ssmo_normals4(seed, tag, i, n, e, _dp(z))
    return z


def stream_normal(seed: int, i: int, e: int, q: int) -> float:
    """Normal q of the Brownian stream of particle i, ensemble e (component q % 4 of block q / 4)."""
    return float(_load().ssmo_stream_normal(seed, i, e, q))


def brownian(seed: int, d: int, i: int, e: int, n0: int, r: int, h_fine: float) -> np.ndarray:
    """Increment of particle i over fine steps n0 .. n0+r-1: [d]."""
    dW = np.zeros(d)
    _load().ssmo_brownian(seed, d, i, e, n0, r, h_fine, _dp(dW))
    return dW


# ---------------------------------------------------------------- scheme pieces
def implicit(x, h, rho=0.0, a=1.0, kappa=0.0, lam=0.0, xbar=None, m2=0.0, max_iter=64):
    """Implicit step (2.3) for one particle: returns (y, newton_iterations)."""
    lib = _load()
    x = _f64(np.atleast_1d(x))
    d = x.shape[0]
    y = np.zeros(d)
    xb = _f64(np.zeros(d) if xbar is None else np.atleast_1d(xbar))
    it = lib.ssmo_implicit(d, _dp(x), h, rho, a, kappa, lam, _dp(xb), m2, max_iter, _dp(y))
    _check(it, "implicit")
    return y, it


def pair_sum(Y: np.ndarray, ell: float) -> np.ndarray:
    """(1/N) sum_j (Y^j - Y^i) exp(-|Y^i - Y^j|^2 / (2 ell^2)); Y is [d][N]."""
    lib = _load()
    Y = _f64(np.atleast_2d(Y))
    d, N = Y.shape
    K = np.zeros_like(Y)
    lib.ssmo_pair_sum(d, N, _dp(Y), ell, _dp(K))
    return K


def pair_sum_at(Y: np.ndarray, ell: float, idx) -> np.ndarray:
    """The pairwise part at targets ``idx`` only: [d][len(idx)]."""
    lib = _load()
    Y = _f64(np.atleast_2d(Y))
    d, N = Y.shape
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    K = np.zeros((d, idx.size))
    lib.ssmo_pair_sum_at(d, N, _dp(Y), ell, idx.size, idx.ctypes.data_as(C.POINTER(C.c_int64)), _dp(K))
    return K


def drift(Y: np.ndarray, c0: float, lam: float, g: float, ell: float) -> np.ndarray:
    """b(Y^i, mu_Y) for every particle; Y is [d][N]."""
    lib = _load()
    Y = _f64(np.atleast_2d(Y))
    d, N = Y.shape
    B = np.zeros_like(Y)
    lib.ssmo_drift(d, N, _dp(Y), c0, lam, g, ell, _dp(B))
    return B


def _cfg(w: dict, keep: list):
    d = int(w["d"])
    systems = w["systems"]
    Ns = np.array([int(s[0]) for s in systems], dtype=np.int64)
    ens = np.array([int(s[1]) for s in systems], dtype=np.int32)
    hs = np.array([float(s[2]) for s in systems], dtype=np.float64)
    keep += [Ns, ens, hs]
    c = _Cfg()
    c.d, c.n_sys = d, len(systems)
    c.N = Ns.ctypes.data_as(C.POINTER(C.c_int64))
    c.ens = ens.ctypes.data_as(C.POINTER(C.c_int32))
    c.h = hs.ctypes.data_as(C.POINTER(C.c_double))
    c.T, c.h_fine, c.seed = float(w["T"]), float(w["h_fine"]), int(w["seed"])
    v, b, s = w["v"], w["b"], w["sigma"]
    c.v_rho, c.v_a = float(v.get("rho", 0.0)), float(v.get("a", 0.0))
    c.v_kappa, c.v_lam = float(v.get("kappa", 0.0)), float(v.get("lam", 0.0))
    c.b_c0, c.b_lam = float(b.get("c0", 0.0)), float(b.get("lam", 0.0))
    c.b_g, c.b_ell = float(b.get("g", 0.0)), float(b.get("ell", 1.0))
    for k in range(d):
        c.s0[k] = float(s["s0"][k]); c.s1[k] = float(s["s1"][k]); c.s2[k] = float(s["s2"][k])
        c.x0_mean[k] = float(w["x0_mean"][k]); c.x0_std[k] = float(w["x0_std"][k])
    c.newton_max_iter = int(w.get("newton_max_iter", 64))
    c.allow_unstable_h = int(bool(w.get("allow_unstable_h", False)))
    # extensions: component-wise cubic in v, b += b_const + b_mat y + b_mean o ybar
    c.v_componentwise = int(bool(v.get("componentwise", False)))
    ak, bc, bm, bmean = v.get("a_k"), b.get("const"), b.get("mat"), b.get("mean")
    for k in range(d):
        c.v_ak[k] = float(ak[k]) if ak is not None else 0.0
        c.b_const[k] = float(bc[k]) if bc is not None else 0.0
        c.b_mean[k] = float(bmean[k]) if bmean is not None else 0.0
        for l in range(d):
            c.b_mat[k * MAX_D + l] = float(bm[k][l]) if bm is not None else 0.0
    return c


def init_state(w: dict, ens: int, N: int) -> np.ndarray:
    """X_0 of one system, [d][N]."""
    lib = _load()
    keep = []
    c = _cfg(w, keep)
    X = np.zeros((c.d, N))
    lib.ssmo_init_state(C.byref(c), ens, N, _dp(X))
    return X


def step(w: dict, ens: int, h: float, n: int, X: np.ndarray):
    """One SSM step of one system from X_n (not modified); returns (X_{n+1}, Y*_n)."""
    lib = _load()
    keep = []
    c = _cfg(w, keep)
    X = _f64(np.atleast_2d(X)).copy()
    Y = np.zeros_like(X)
    st = lib.ssmo_step(C.byref(c), ens, X.shape[1], h, n, _dp(X), _dp(Y))
    _check(st, "step")
    return X, Y


def step_at(w: dict, ens: int, h: float, n: int, X: np.ndarray, idx) -> np.ndarray:
    """One SSM step of one system from X_n, evaluated at the particles ``idx``
    only: X_{n+1} at them, [d][len(idx)] (Y* is solved for every particle; the
    O(N^2) term only at the sampled ones)."""
    lib = _load()
    keep = []
    c = _cfg(w, keep)
    X = _f64(np.atleast_2d(X))
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    out = np.zeros((X.shape[0], idx.size))
    st = lib.ssmo_step_at(C.byref(c), ens, X.shape[1], h, n, _dp(X), idx.size,
                          idx.ctypes.data_as(C.POINTER(C.c_int64)), _dp(out))
    _check(st, "step_at")
    return out


def run(w: dict, stop_after: int = 0):
    """Run every system of ``w`` from 0 to T (or ``stop_after`` steps); list of [d][N_s]."""
    lib = _load()
    keep = []
    c = _cfg(w, keep)
    Ns = [int(s[0]) for s in w["systems"]]
    X = np.zeros(sum(Ns) * c.d)
    steps = np.zeros(len(Ns), dtype=np.int64)
    st = lib.ssmo_run(C.byref(c), stop_after, _dp(X), steps.ctypes.data_as(C.POINTER(C.c_int64)))
    _check(st, "run")
    out, off = [], 0
    for N in Ns:
        out.append(X[off:off + c.d * N].reshape(c.d, N).copy())
        off += c.d * N
    return out


def moments(X: np.ndarray):
    """(mean_k, var_k) with the 1/N normalisation, two passes."""
    lib = _load()
    X = _f64(np.atleast_2d(X))
    d, N = X.shape
    m, v = np.zeros(d), np.zeros(d)
    lib.ssmo_moments(d, N, _dp(X), _dp(m), _dp(v))
    return m, v


# ---------------------------------------------------------------- learned surrogate (not in the paper)
def rff_omegas(seed: int, d: int, K: int, ell: float) -> np.ndarray:
    """Frequencies omega_k = Z(3, k, 0, 0)[:d] / ell, [K][d]."""
    lib = _load()
    om = np.zeros((K, d))
    lib.ssmo_rff_omegas(seed, d, K, ell, _dp(om))
    return om


def rff_moments(Y: np.ndarray, omega: np.ndarray) -> np.ndarray:
    """[cos moments (K), sin moments (K)] of the empirical measure of Y [d][N]."""
    lib = _load()
    Y = _f64(np.atleast_2d(Y))
    om = _f64(omega)
    K = om.shape[0]
    m = np.zeros(2 * K)
    lib.ssmo_rff_moments(Y.shape[0], Y.shape[1], _dp(Y), K, _dp(om), _dp(m))
    return m


def mlp_num_params(n_in: int, H: int, n_out: int) -> int:
    return int(_load().ssmo_mlp_num_params(n_in, H, n_out))


def mlp_forward(params, X, n_in: int, H: int, n_out: int) -> np.ndarray:
    lib = _load()
    p = _f64(params)
    X = _f64(X).reshape(-1, n_in)
    Y = np.zeros((X.shape[0], n_out))
    lib.ssmo_mlp_forward(n_in, H, n_out, _dp(p), X.shape[0], _dp(X), _dp(Y))
    return Y


def mlp_loss_grad(params, X, T, n_in: int, H: int, n_out: int):
    """(loss, gradient) of L = (1/B) sum_b |MLP(X_b) - T_b|^2."""
    lib = _load()
    p = _f64(params)
    X = _f64(X).reshape(-1, n_in)
    T = _f64(T).reshape(-1, n_out)
    g = np.zeros_like(p)
    loss = lib.ssmo_mlp_loss_grad(n_in, H, n_out, _dp(p), X.shape[0], _dp(X), _dp(T), _dp(g))
    return float(loss), g


def num_threads() -> int:
    return int(_load().ssmo_num_threads())


def set_num_threads(n: int) -> None:
    _load().ssmo_set_num_threads(int(n))


# ---------------------------------------------------------------- error statistics (Section 3)
def strong_error(X: np.ndarray, X_ref: np.ndarray) -> float:
    """epsilon_2 of Section 3: ((1/N) sum_j |X^j - X_ref^j|^2)^(1/2); arrays [d][N] or lists of them."""
    if isinstance(X, (list, tuple)):
        num = sum(float(np.sum((np.asarray(a) - np.asarray(b)) ** 2)) for a, b in zip(X, X_ref))
        cnt = sum(np.asarray(a).shape[-1] for a in X)
        return float(np.sqrt(num / cnt))
    D = np.atleast_2d(X) - np.atleast_2d(X_ref)
    return float(np.sqrt(np.sum(D * D) / D.shape[1]))


def weak_error(X: np.ndarray, X_ref: np.ndarray) -> float:
    """epsilon_1 of Section 3: |(1/N) sum_j (X^j - X_ref^j)|_2; arrays [d][N] or
    lists of them (the mean then runs over the particles of all systems)."""
    if isinstance(X, (list, tuple)):
        D = np.concatenate([np.atleast_2d(a) - np.atleast_2d(b) for a, b in zip(X, X_ref)], axis=1)
    else:
        D = np.atleast_2d(X) - np.atleast_2d(X_ref)
    return float(np.linalg.norm(D.mean(axis=1)))


def ols_slope(hs, errs) -> float:
    """Least-squares slope of log2(err) against log2(h)."""
    x = np.log2(np.asarray(hs, dtype=np.float64))
    y = np.log2(np.asarray(errs, dtype=np.float64))
    x0 = x - x.mean()
    return float(np.sum(x0 * (y - y.mean())) / np.sum(x0 * x0))
