"""Python front end of libssm: the split-step method (SSM) of arXiv:2105.09688
(Section 2.2, eqs. (2.3)-(2.4)) for N-particle McKean-Vlasov systems on one
MI355X.  Thin ctypes marshalling; PyTorch provides device memory and streams."""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib
from ._lib import SSM_FP32, SSM_FP32_KAHAN, SSM_FP64, check

PRECISIONS = {"fp64": SSM_FP64, "fp32": SSM_FP32, "fp32_kahan": SSM_FP32_KAHAN}


def _torch():
    import torch
    return torch


def _stream_ptr(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


class SSM:
    """One context: n systems advanced together (see include/ssm.h).

    ``workload`` is the dict of ``paper_2105_09688_amd.workloads``."""

    def __init__(self, workload: dict, precision: str = "fp64", stream=None,
                 targets_per_lane: int = 0, sources_per_item: int = 0, graphs: bool = False,
                 pair_scheme: str = "default", kahan_span: int = 0, jside_band_groups: int = 0,
                 persistent: int = 0):
        lib = _lib.load()
        w = workload
        d = int(w["d"])
        systems = w["systems"]
        self.d = d
        self.N = [int(s[0]) for s in systems]
        self._Ns = (C.c_int64 * len(systems))(*self.N)
        self._ens = (C.c_int32 * len(systems))(*[int(s[1]) for s in systems])
        self._hs = (C.c_double * len(systems))(*[float(s[2]) for s in systems])
        c = _lib.Config()
        c.d, c.n_sys = d, len(systems)
        c.N, c.ens, c.h = self._Ns, self._ens, self._hs
        c.T, c.h_fine, c.seed = float(w["T"]), float(w["h_fine"]), int(w["seed"])
        c.precision = PRECISIONS[precision]
        v, b, s = w["v"], w["b"], w["sigma"]
        c.v_rho, c.v_a = float(v.get("rho", 0.0)), float(v.get("a", 0.0))
        c.v_kappa, c.v_lam = float(v.get("kappa", 0.0)), float(v.get("lam", 0.0))
        c.b_c0, c.b_lam = float(b.get("c0", 0.0)), float(b.get("lam", 0.0))
        c.b_g, c.b_ell = float(b.get("g", 0.0)), float(b.get("ell", 1.0))
        for k in range(d):
            c.s0[k], c.s1[k], c.s2[k] = float(s["s0"][k]), float(s["s1"][k]), float(s["s2"][k])
            c.x0_mean[k], c.x0_std[k] = float(w["x0_mean"][k]), float(w["x0_std"][k])
        c.newton_max_iter = int(w.get("newton_max_iter", 0))
        c.allow_unstable_h = int(bool(w.get("allow_unstable_h", False)))
        c.stream = _stream_ptr(stream)
        c.targets_per_lane = int(targets_per_lane)
        c.sources_per_item = int(sources_per_item)
        c.graphs = 1 if graphs else 0
        c.pair_scheme = {"default": 0, "ordered": 1, "symmetric": 2}[pair_scheme]
        c.kahan_span = int(kahan_span)  # 1: every pair term compensated (fp32_kahan, ordered pairs)
        c.jside_band_groups = int(jside_band_groups)  # symmetric scheme: j-side rows in bands of this many groups
        c.persistent = int(persistent)  # small systems in one launch per step call: 0 default, 1 on, -1 off
        # coefficient extensions: component-wise cubic in v, b += b_const + b_mat y + b_mean o ybar
        c.v_componentwise = int(bool(v.get("componentwise", False)))
        ak, bc, bm, bmean = v.get("a_k"), b.get("const"), b.get("mat"), b.get("mean")
        for k in range(d):
            c.v_ak[k] = float(ak[k]) if ak is not None else 0.0
            c.b_const[k] = float(bc[k]) if bc is not None else 0.0
            c.b_mean[k] = float(bmean[k]) if bmean is not None else 0.0
            for l in range(d):
                c.b_mat[k * _lib.MAX_D + l] = float(bm[k][l]) if bm is not None else 0.0
        self._cfg = c
        h = C.c_void_p()
        check(lib.ssm_init(C.byref(c), C.byref(h)))
        self._h = h
        self.precision = precision

    # -- lifecycle ---------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            _lib.load().ssm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- stepping ----------------------------------------------------------
    def step(self, n_ticks: int = 1):
        check(_lib.load().ssm_step(self._h, int(n_ticks)))

    def run(self):
        check(_lib.load().ssm_run(self._h))

    def sync(self):
        check(_lib.load().ssm_sync(self._h))

    # -- outputs -----------------------------------------------------------
    def moments(self, sys: int = 0):
        m = np.zeros(self.d)
        v = np.zeros(self.d)
        check(_lib.load().ssm_moments(self._h, sys, m.ctypes.data_as(C.POINTER(C.c_double)),
                                      v.ctypes.data_as(C.POINTER(C.c_double))))
        return m, v

    def state(self, sys: int = 0, which: str = "x"):
        out = np.zeros((self.d, self.N[sys]))
        step = C.c_int64()
        check(_lib.load().ssm_get_state(self._h, sys, 0 if which == "x" else 1,
                                        out.ctypes.data_as(C.POINTER(C.c_double)), C.byref(step)))
        return out

    def states(self, which: str = "x"):
        return [self.state(s, which) for s in range(len(self.N))]

    def state_step(self, sys: int = 0, which: str = "x"):
        """(state [d][N] as float64, steps system sys has taken) (ssm_get_state)."""
        out = np.zeros((self.d, self.N[sys]))
        step = C.c_int64()
        check(_lib.load().ssm_get_state(self._h, sys, 0 if which == "x" else 1,
                                        out.ctypes.data_as(C.POINTER(C.c_double)), C.byref(step)))
        return out, step.value

    def set_state(self, sys: int, X, step: int = -1) -> None:
        """X of system sys (ssm_set_state); step >= 0 also moves the context to
        that step of system sys (a resume on the same Brownian paths)."""
        X = np.ascontiguousarray(X, dtype=np.float64).reshape(self.d, self.N[sys])
        check(_lib.load().ssm_set_state(self._h, sys, X.ctypes.data_as(C.POINTER(C.c_double)), int(step)))

    def surrogate_train(self, n_samples: int, n_ens: int = 2, ens0: int = 1, N: int = 0, snapshots: int = 32,
                        steps: int = 4000, batch: int = 2048, lr: float = 1e-3, seed: int = 0, init=None):
        """Train the surrogate inside the library on exact runs of n_ens systems
        like system 0 and load it (ssm_surrogate_train).  Returns (weights,
        loss history) as numpy float32 arrays."""
        cfg = _lib.SurrTrainCfg()
        cfg.n_ens, cfg.ens0, cfg.N, cfg.n_samples = int(n_ens), int(ens0), int(N), int(n_samples)
        cfg.snapshots, cfg.seed = int(snapshots), int(seed)
        cfg.train.steps, cfg.train.batch, cfg.train.lr, cfg.train.seed = int(steps), int(batch), float(lr), int(seed)
        out = np.zeros(mlp_num_params(self.d), dtype=np.float32)
        hist = np.zeros(int(steps), dtype=np.float32)
        ini = None
        if init is not None:
            ini = np.ascontiguousarray(init, dtype=np.float32)
            if ini.size != out.size:
                raise ValueError(f"init needs {out.size} parameters")
        check(_lib.load().ssm_surrogate_train(self._h, C.byref(cfg), None if ini is None else ini.ctypes.data,
                                              out.ctypes.data, hist.ctypes.data))
        return out, hist

    # -- the state in caller-owned device memory -----------------------------
    def state_layout(self):
        """(P, offsets, element bytes) of the device state X (ssm_state_layout)."""
        P = C.c_int64()
        offs = (C.c_int64 * len(self.N))()
        e = C.c_int32()
        check(_lib.load().ssm_state_layout(self._h, C.byref(P), offs, C.byref(e)))
        return P.value, list(offs), e.value

    def bind_state(self, buf=None):
        """Make a CUDA tensor [d][P] of the storage dtype the context's X
        (ssm_bind_state); a new one is allocated when buf is None.  Returns it;
        the context keeps a reference, so the memory outlives the context."""
        torch = _torch()
        P, offs, e = self.state_layout()
        dt = torch.float64 if e == 8 else torch.float32
        if buf is None:
            buf = torch.empty((self.d, P), dtype=dt, device="cuda")
        if buf.dtype != dt or not buf.is_cuda or not buf.is_contiguous() or tuple(buf.shape) != (self.d, P):
            raise ValueError(f"state buffer must be a contiguous CUDA tensor {dt} of shape ({self.d}, {P})")
        check(_lib.load().ssm_bind_state(self._h, C.c_void_p(buf.data_ptr()), buf.numel() * buf.element_size()))
        self._bound, self._offs = buf, offs
        return buf

    def state_view(self, sys: int = 0):
        """View [d][N_s] of system sys in the bound state tensor (after bind_state)."""
        return self._bound[:, self._offs[sys]:self._offs[sys] + self.N[sys]]

    def refresh(self, sys: int = -1) -> None:
        """Recompute Y* after X was changed through the bound tensor (ssm_state_refresh)."""
        check(_lib.load().ssm_state_refresh(self._h, int(sys)))

    def rmse(self, other: "SSM"):
        per = np.zeros(len(self.N))
        r = C.c_double()
        check(_lib.load().ssm_rmse(self._h, other._h, per.ctypes.data_as(C.POINTER(C.c_double)), C.byref(r)))
        return r.value, per

    def sqdiff(self, sys: int, other: "SSM", other_sys: int) -> float:
        """sum_i |X_self^i - X_other^i|^2 over one system of each context."""
        r = C.c_double()
        check(_lib.load().ssm_sqdiff(self._h, sys, other._h, other_sys, C.byref(r)))
        return r.value

    # -- learned surrogate ----------------------------------------------------
    def surrogate_load(self, master) -> None:
        """Load FP32 master weights (numpy or CPU tensor, flat layout of include/ssm.h)."""
        m = np.ascontiguousarray(np.asarray(master, dtype=np.float32).ravel())
        check(_lib.load().ssm_surrogate_load(self._h, m.ctypes.data, m.size))

    def surrogate_enable(self, check_every: int = 16, tol: float = 1e-3, mode: str = "gain",
                         recheck: bool = False) -> None:
        """mode "gain": g (s - mean s); "residual": (s - mean s) + the residual of the last check.
        recheck: during a fallback every tick on which all systems step is a check too."""
        modes = {"gain": 0, "residual": 1}
        if mode not in modes:
            raise ValueError(f"mode must be one of {sorted(modes)}")
        check(_lib.load().ssm_surrogate_enable(self._h, int(check_every), float(tol), modes[mode]))
        check(_lib.load().ssm_surrogate_recheck(self._h, 1 if recheck else 0))

    def surrogate_predict(self, sys: int = 0):
        """(network output s [d][N] float64, RFF moments [2K] float32) at the
        current Y* of system sys, from the surrogate tick's kernels."""
        out = np.zeros((self.d, self.N[sys]))
        mom = np.zeros(32, dtype=np.float32)
        check(_lib.load().ssm_surrogate_predict(self._h, sys, out.ctypes.data_as(C.POINTER(C.c_double)),
                                                mom.ctypes.data))
        return out, mom

    def surrogate_samples(self, n: int, seed: int, sys: int = 0):
        """(U [n][d+32], T [n][d]) float32 device tensors from the current state."""
        torch = _torch()
        U = torch.empty((n, self.d + 32), dtype=torch.float32, device="cuda")
        T = torch.empty((n, self.d), dtype=torch.float32, device="cuda")
        check(_lib.load().ssm_surrogate_samples(self._h, sys, n, seed, U.data_ptr(), T.data_ptr()))
        return U, T

    def profile(self, enable: bool = True, every: int = 1) -> None:
        """Time the pair and update launches of every `every`-th tick with HIP events."""
        check(_lib.load().ssm_profile(self._h, int(every) if enable else 0))

    def info(self) -> dict:
        i = _lib.Info()
        check(_lib.load().ssm_info(self._h, C.byref(i)))
        out = {f: getattr(i, f) for f, _ in i._fields_}
        out["surr_gain"] = list(out["surr_gain"])[: self.d]
        out["pair_scheme"] = "symmetric" if out.pop("symmetric") else "ordered"
        return out


# -------------------------------------------------------------------------- kernel-level calls
def _cur_stream():
    return _torch().cuda.current_stream().cuda_stream


def pair_sum(Y, ell: float, precision: str = "fp64"):
    """K[k][i] = (1/N) sum_j (Y_k^j - Y_k^i) exp(-|Y^i - Y^j|^2/(2 ell^2)) for a device tensor Y [d][N]
    (float64 for 'fp64', float32 otherwise).  Returns a float64 device tensor [d][N]."""
    torch = _torch()
    lib = _lib.load()
    prec = PRECISIONS[precision]
    want = torch.float64 if prec == SSM_FP64 else torch.float32
    if Y.dtype != want or not Y.is_cuda or Y.dim() != 2:
        raise ValueError(f"Y must be a 2-D CUDA tensor of {want}")
    Y = Y.contiguous()
    d, N = Y.shape
    K = torch.empty((d, N), dtype=torch.float64, device=Y.device)
    nbytes = lib.ssm_pair_workspace_bytes(d, N, prec)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=Y.device)
    check(lib.ssm_pair_sum(d, N, prec, Y.data_ptr(), float(ell), K.data_ptr(), ws.data_ptr(),
                           nbytes, _cur_stream()))
    return K


def implicit_solve(X, h: float, rho=0.0, a=1.0, kappa=0.0, lam=0.0, xbar=None, m2=0.0, max_iter=64):
    """Y = F_h(X) of (2.3) for a float64 device tensor X [d][N]; returns (Y, iterations)."""
    torch = _torch()
    lib = _lib.load()
    if X.dtype != torch.float64 or not X.is_cuda or X.dim() != 2:
        raise ValueError("X must be a 2-D float64 CUDA tensor")
    X = X.contiguous()
    d, N = X.shape
    Y = torch.empty_like(X)
    it = torch.empty(N, dtype=torch.int32, device=X.device)
    xb = np.zeros(d) if xbar is None else np.ascontiguousarray(xbar, dtype=np.float64)
    check(lib.ssm_implicit_solve(d, N, X.data_ptr(), h, rho, a, kappa, lam,
                                 xb.ctypes.data_as(C.POINTER(C.c_double)), m2, max_iter,
                                 Y.data_ptr(), it.data_ptr(), _cur_stream()))
    return Y, it


def brownian(d: int, N: int, seed: int, ens: int, n0: int, r: int, h_fine: float, device="cuda"):
    """dW[k][i] = sqrt(h_fine) sum_{m<r} Z(0, i, n0+m, ens)_k as a float64 device tensor."""
    torch = _torch()
    dW = torch.empty((d, N), dtype=torch.float64, device=device)
    check(_lib.load().ssm_brownian(d, N, seed, ens, n0, r, h_fine, dW.data_ptr(), _cur_stream()))
    return dW


def philox_blocks(ctr, key, count: int, device="cuda"):
    """Philox4x64-10 blocks of counters (ctr[0]+q, ctr[1], ctr[2], ctr[3]), q < count; int64 view [count, 4]."""
    torch = _torch()
    out = torch.empty((count, 4), dtype=torch.int64, device=device)
    c = [int(v) & (2 ** 64 - 1) for v in ctr]
    k = [int(v) & (2 ** 64 - 1) for v in key]
    check(_lib.load().ssm_philox_blocks(c[0], c[1], c[2], c[3], k[0], k[1], count, out.data_ptr(), _cur_stream()))
    return out


# -------------------------------------------------------------------------- surrogate network
def mlp_num_params(d: int) -> int:
    return int(_lib.load().ssm_mlp_num_params(d))


def mlp_init(d: int, seed: int = 0):
    """Seeded initial FP32 master weights (uniform +-sqrt(6/(fan_in+fan_out)) per matrix, zero biases)."""
    rng = np.random.Generator(np.random.Philox(key=seed + 5))
    shapes = [(64, 2 * d + 32), (64, 64), (64, 64), (d, 64)]
    parts = []
    for (o, i) in shapes:
        lim = np.sqrt(6.0 / (i + o))
        parts.append(rng.uniform(-lim, lim, size=o * i))
        parts.append(np.zeros(o))
    out = np.concatenate(parts).astype(np.float32)
    assert out.size == mlp_num_params(d)
    return out


def mlp_forward(d: int, master, U):
    """Network output for raw device float32 rows U [n][d+32] = [y, moments]; master: device float32."""
    torch = _torch()
    out = torch.empty((U.shape[0], d), dtype=torch.float32, device=U.device)
    check(_lib.load().ssm_mlp_forward(d, master.data_ptr(), U.contiguous().data_ptr(), U.shape[0],
                                      out.data_ptr(), _cur_stream()))
    return out


def mlp_forward_noalloc(d: int, master, U, out):
    """mlp_forward into a caller-allocated float32 device tensor out [n][d], with
    no allocation in the library (ssm_mlp_forward_noalloc); asynchronous on the
    current stream."""
    check(_lib.load().ssm_mlp_forward_noalloc(d, master.data_ptr(), U.data_ptr(), U.shape[0], out.data_ptr(),
                                              _cur_stream()))
    return out


def mlp_loss_grad(d: int, master, U, T):
    """(loss, grad) for the rows of U, T in order (row count a multiple of 64)."""
    torch = _torch()
    g = torch.zeros_like(master)
    loss = C.c_double()
    check(_lib.load().ssm_mlp_loss_grad(d, master.data_ptr(), U.contiguous().data_ptr(), T.contiguous().data_ptr(),
                                        U.shape[0], g.data_ptr(), C.byref(loss), _cur_stream()))
    return loss.value, g


def mlp_train(d: int, master, U, T, steps: int, batch: int = 4096, lr: float = 1e-3, seed: int = 0):
    """Adam on the device master weights (in place); returns the per-step loss history."""
    cfg = _lib.TrainCfg()
    cfg.steps, cfg.batch, cfg.lr, cfg.seed = int(steps), int(batch), float(lr), int(seed)
    hist = np.zeros(int(steps), dtype=np.float32)
    check(_lib.load().ssm_mlp_train(d, U.contiguous().data_ptr(), T.contiguous().data_ptr(), U.shape[0],
                                    C.byref(cfg), master.data_ptr(), hist.ctypes.data, _cur_stream()))
    return hist
