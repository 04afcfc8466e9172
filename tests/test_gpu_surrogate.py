"""Learned surrogate of the pairwise term (an extension, not in the paper):
its kernels against the FP64 oracle, and its use inside the SSM step."""
import sys

import numpy as np
import pytest

import errstats
import oracle
from paper_2105_09688_amd import workloads as W

pytestmark = pytest.mark.gpu
D = 2
IN = D + 32          # raw rows handed to the library: [y, moments]
IN_NET = 2 * D + 32  # network inputs: [hi(y), lo(y), moments]


def _say(msg):
    print(f"[gpu-surrogate] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    return torch


def _bf16(x):
    """Round float values to bfloat16 (nearest even), returned as float64."""
    import torch
    return torch.tensor(np.asarray(x, dtype=np.float32)).to(torch.bfloat16).to(torch.float64).numpy()


def _kernel_params(p):
    """The parameters as the kernels hold them: weight matrices rounded to
    BF16, biases kept in float32; float64."""
    out = np.asarray(p, dtype=np.float32).astype(np.float64)
    off = 0
    for (o, i) in [(64, IN_NET), (64, 64), (64, 64), (D, 64)]:
        out[off:off + o * i] = _bf16(out[off:off + o * i])
        off += o * i + o
    return out


def _expand(U, round_moments=True):
    """Network inputs of raw rows as the kernels form them: hi(y) = bf16(y),
    lo(y) = bf16(y - hi(y)), then the moments, bf16-rounded as the training
    kernels take them or (round_moments=False) as the float32 values that the
    split-precision inference carries to about 16 bits; float64."""
    U = np.asarray(U, dtype=np.float32)
    hi = _bf16(U[:, :D])
    lo = _bf16(U[:, :D].astype(np.float64) - hi)
    m = _bf16(U[:, D:]) if round_moments else U[:, D:].astype(np.float64)
    return np.concatenate([hi, lo, m], axis=1)


def _small_w(N=4096, T=2.0 ** -4):
    w = W.surrogate_d2(N=N, h=2.0 ** -9, h_fine=2.0 ** -9)
    w["T"] = T
    return w


def test_mfma_forward_matches_oracle(torch_cuda):
    """Inference (BF16 weights, activations split into BF16 hi + lo parts)
    against the oracle's FP64 forward at the same parameters and unrounded
    moments: relative error <= 5e-5 (plain BF16 activations would be at
    about 3e-3 on these rows)."""
    torch = torch_cuda
    from paper_2105_09688_amd.ssm import mlp_forward, mlp_init
    p = mlp_init(D, seed=1)
    p += np.random.default_rng(3).normal(size=p.size).astype(np.float32) * 0.05  # nonzero biases
    rng = np.random.default_rng(2)
    U = rng.normal(size=(1000, IN)).astype(np.float32)
    _say("mlp forward")
    got = mlp_forward(D, torch.tensor(p, device="cuda"), torch.tensor(U, device="cuda")).cpu().numpy()
    ref = oracle.mlp_forward(_kernel_params(p), _expand(U, round_moments=False), IN_NET, 64, D)
    rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    _say(f"forward rel err {rel:.3e}")
    assert rel <= 5e-5


# Element-wise bar of the split-precision inference against the oracle's
# FP64 forward at the same (BF16-rounded) weights: each activation enters the
# matrix cores as hi + lo BF16 parts (about 16 significant bits, relative
# rounding <= 2^-17), products accumulate in FP32 over K = 64, and four layers
# compound it; at unit-size outputs this is a few 1e-6 absolute.  The bar
# max_i |got_i - ref_i| / max(1, |ref_i|) <= 5e-5 leaves an order of magnitude
# of room and is still 60x below the error of plain BF16 activations (about
# 3e-3, which the test also shows the bar would catch).
ELEMENT_BAR = 5e-5


def _elem_err(got, ref):
    return float(np.max(np.abs(got - ref) / np.maximum(1.0, np.abs(ref))))


@pytest.mark.parametrize("n", [1000, 4099])
def test_mlp_apply_elementwise_matches_oracle(torch_cuda, n):
    """ssm_mlp_forward (k_mlp_apply) on n raw rows (ragged: not a multiple of
    the 16-row tile or the 64-row block) against oracle.mlp_forward element
    by element, with the moments passed unrounded (the split inference carries
    them to about 16 bits)."""
    torch = torch_cuda
    from paper_2105_09688_amd.ssm import mlp_forward, mlp_init
    p = mlp_init(D, seed=11)
    p += np.random.default_rng(12).normal(size=p.size).astype(np.float32) * 0.05
    rng = np.random.default_rng(13)
    U = np.concatenate([rng.normal(size=(n, D)) * 1.5, rng.uniform(-1, 1, size=(n, 32))], axis=1).astype(np.float32)
    got = mlp_forward(D, torch.tensor(p, device="cuda"), torch.tensor(U, device="cuda")).cpu().numpy()
    ref = oracle.mlp_forward(_kernel_params(p), _expand(U, round_moments=False), IN_NET, 64, D)
    err = _elem_err(got, ref)
    # what plain BF16 activations would give: the bar separates the two
    ref_bf = oracle.mlp_forward(_kernel_params(p), _expand(U), IN_NET, 64, D)
    _say(f"mlp_apply n={n}: element-wise err {err:.3e} (moments rounded to BF16: {_elem_err(ref_bf, ref):.3e})")
    assert got.shape == (n, D)
    assert err <= ELEMENT_BAR


@pytest.mark.parametrize("precision", ["fp64", "fp32_kahan"])
def test_mlp_infer_in_step_matches_oracle_elementwise(torch_cuda, precision):
    """The kernels a surrogate tick runs (RFF moments, then k_mlp_infer over
    the context's SoA Y*, stored per component) in one context of two systems
    of ragged sizes (1000 and 4099, ensembles 0 and 1), each set to the
    oracle's X_3 of its own run (ssm_set_state at step 3), so that Y* is the
    oracle's F_h(X_3).  Against the oracle:
      - the RFF moments of mu^Y per system (FP32 sin/cos in the kernel):
        max abs difference <= 2e-6;
      - the network output per particle and component, element-wise against
        oracle.mlp_forward at the oracle's own Y* and moments: <= 1e-4 (the
        element bar plus the moments' 2e-6 through the first layer);
      - the same against oracle.mlp_forward at the GPU's moments: the element bar."""
    from paper_2105_09688_amd.ssm import SSM, mlp_init
    h = 2.0 ** -9
    w = W.surrogate_d2(N=1000, h=h, h_fine=h)
    w["systems"] = [(1000, 0, h), (4099, 1, h)]
    w["T"] = 8 * h
    p = mlp_init(D, seed=21)
    p += np.random.default_rng(22).normal(size=p.size).astype(np.float32) * 0.05
    om = oracle.rff_omegas(w["seed"], D, 16, w["b"]["ell"])
    ref_states = []
    for (N, e, _h) in w["systems"]:
        X = oracle.init_state(w, e, N)
        for n in range(3):
            X, _ = oracle.step(w, e, h, n, X)
        _, Y = oracle.step(w, e, h, 3, X)
        ref_states.append((X, Y))
    with SSM(w, precision=precision) as s:
        for k, (X, _Y) in enumerate(ref_states):
            s.set_state(k, X, step=3)
        s.surrogate_load(p)
        for k, (N, e, _h) in enumerate(w["systems"]):
            X, Y = ref_states[k]
            Yg = s.state(k, "y")
            out, mom = s.surrogate_predict(k)
            ydiff = float(np.max(np.abs(Yg - Y)))
            mref = oracle.rff_moments(Y, om)
            merr = float(np.max(np.abs(mom.astype(np.float64) - mref)))
            rows_o = np.concatenate([Y.T, np.broadcast_to(mref, (N, 32))], axis=1)
            ref_o = oracle.mlp_forward(_kernel_params(p), _expand(rows_o, round_moments=False), IN_NET, 64, D)
            rows_g = np.concatenate([Yg.T, np.broadcast_to(mom.astype(np.float64), (N, 32))], axis=1)
            ref_g = oracle.mlp_forward(_kernel_params(p), _expand(rows_g, round_moments=False), IN_NET, 64, D)
            e_o, e_g = _elem_err(out.T, ref_o), _elem_err(out.T, ref_g)
            _say(f"infer {precision} sys {k} N={N}: |Y* - oracle| {ydiff:.2e}, moments {merr:.2e}, "
                 f"output vs oracle (own moments) {e_o:.3e}, (GPU moments) {e_g:.3e}")
            assert out.shape == (D, N)
            assert ydiff <= (1e-14 if precision == "fp64" else 1e-6)
            assert merr <= 2e-6
            assert e_o <= 1e-4
            assert e_g <= ELEMENT_BAR


def test_adam_steps_match_the_adam_update(torch_cuda):
    """ssm_mlp_train's optimizer (k_adam) against Adam's update (Kingma & Ba,
    bias-corrected), for one step and for the second step of a two-step call:
    one distinct training row, so every minibatch row is that row and each
    step's gradient is ssm_mlp_loss_grad at the current weights on 64 copies
    of it.  m_t = b1 m + (1 - b1) g, v_t = b2 v + (1 - b2) g^2,
    w -= lr (m_t / (1 - b1^t)) / (sqrt(v_t / (1 - b2^t)) + eps), evaluated in
    FP64 from the FP32 gradients and weights; element-wise within half an FP32
    ulp of the weight plus 1e-6 lr (the FP32 arithmetic of the update)."""
    torch = torch_cuda
    from paper_2105_09688_amd.ssm import mlp_init, mlp_loss_grad, mlp_train
    p0 = mlp_init(D, seed=31)
    p0 += np.random.default_rng(32).normal(size=p0.size).astype(np.float32) * 0.05
    rng = np.random.default_rng(33)
    U1 = rng.normal(size=(1, IN)).astype(np.float32)
    T1 = rng.normal(size=(1, D)).astype(np.float32) * 0.3
    U64, T64 = np.repeat(U1, 64, axis=0), np.repeat(T1, 64, axis=0)
    lr, b1, b2, eps = 1e-2, 0.9, 0.999, 1e-8

    def dev(a):
        return torch.tensor(np.asarray(a, dtype=np.float32), device="cuda")

    def grad(wt):
        return mlp_loss_grad(D, dev(wt), dev(U64), dev(T64))[1].cpu().numpy().astype(np.float64)

    w1 = dev(p0)
    mlp_train(D, w1, dev(U1), dev(T1), steps=1, batch=64, lr=lr, seed=1)
    w1 = w1.cpu().numpy().astype(np.float64)
    g1 = grad(p0)
    m1, v1 = (1 - b1) * g1, (1 - b2) * g1 * g1
    w1_ref = p0.astype(np.float64) - lr * (m1 / (1 - b1)) / (np.sqrt(v1 / (1 - b2)) + eps)
    err1 = float(np.max(np.abs(w1 - w1_ref))) / lr
    w2 = dev(p0)
    mlp_train(D, w2, dev(U1), dev(T1), steps=2, batch=64, lr=lr, seed=2)
    w2 = w2.cpu().numpy().astype(np.float64)
    g2 = grad(w1)  # step 2 starts from step 1's weights (the same kernels, deterministic)
    m2, v2 = b1 * m1 + (1 - b1) * g2, b2 * v1 + (1 - b2) * g2 * g2
    w2_ref = w1 - lr * (m2 / (1 - b1 ** 2)) / (np.sqrt(v2 / (1 - b2 ** 2)) + eps)
    err2 = float(np.max(np.abs(w2 - w2_ref))) / lr
    _say(f"adam: step 1 max |w - w_ref| / lr = {err1:.2e}, step 2 {err2:.2e}; "
         f"mean |update| / lr {np.mean(np.abs(w1 - p0)) / lr:.3f}, {np.mean(np.abs(w2 - w1)) / lr:.3f}")
    # the FP32 weight itself rounds to half an ulp (2^-24 relative), the update's own arithmetic adds 1e-6 lr
    assert np.all(np.abs(w1 - w1_ref) <= 2.0 ** -24 * np.abs(w1_ref) + 1e-6 * lr)
    assert np.all(np.abs(w2 - w2_ref) <= 2.0 ** -24 * np.abs(w2_ref) + 1e-6 * lr)
    assert np.mean(np.abs(w2 - w1)) > 0.1 * lr  # the second step moved the weights


def test_mfma_gradient_matches_oracle(torch_cuda):
    """GPU BF16/FP32 gradient vs the oracle's FP64 back-propagation at the same
    parameters (BF16 weight matrices, float32 biases) and BF16-rounded inputs:
    per-tensor relative error <= 2e-2 and cosine >= 0.999."""
    torch = torch_cuda
    from paper_2105_09688_amd.ssm import mlp_init, mlp_loss_grad
    p = mlp_init(D, seed=3)
    p += np.random.default_rng(4).normal(size=p.size).astype(np.float32) * 0.05  # nonzero biases
    rng = np.random.default_rng(5)
    U = rng.normal(size=(512, IN)).astype(np.float32)
    T = rng.normal(size=(512, D)).astype(np.float32) * 0.3
    _say("mlp gradient")
    loss, g = mlp_loss_grad(D, torch.tensor(p, device="cuda"), torch.tensor(U, device="cuda"),
                            torch.tensor(T, device="cuda"))
    g = g.cpu().numpy().astype(np.float64)
    loss_ref, g_ref = oracle.mlp_loss_grad(_kernel_params(p), _expand(U), T.astype(np.float64), IN_NET, 64, D)
    assert loss == pytest.approx(loss_ref, rel=1e-2)
    sizes = [64 * IN_NET, 64, 64 * 64, 64, 64 * 64, 64, D * 64, D]
    off = 0
    for k, n in enumerate(sizes):
        a, b = g[off:off + n], g_ref[off:off + n]
        rel = np.linalg.norm(a - b) / np.linalg.norm(b)
        cos = float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b)))
        _say(f"tensor {k}: rel {rel:.3e} cos {cos:.6f}")
        assert rel <= 2e-2 and cos >= 0.999, k
        off += n


def test_training_fits_a_smooth_target(torch_cuda):
    torch = torch_cuda
    from paper_2105_09688_amd.ssm import mlp_forward, mlp_init, mlp_train
    rng = np.random.default_rng(6)
    U = rng.normal(size=(20000, IN)).astype(np.float32)
    T = np.stack([np.tanh(U[:, 0] - 0.5 * U[:, 3]), 0.3 * U[:, 1] * U[:, 2]], axis=1).astype(np.float32)
    p = torch.tensor(mlp_init(D, seed=7), device="cuda")
    Ud, Td = torch.tensor(U, device="cuda"), torch.tensor(T, device="cuda")
    _say("training")
    hist = mlp_train(D, p, Ud, Td, steps=1500, batch=1024, lr=3e-3, seed=1)
    assert np.all(np.isfinite(hist))
    first, last = float(np.mean(hist[:20])), float(np.mean(hist[-50:]))
    _say(f"loss {first:.4f} -> {last:.5f}")
    assert last < 0.05 * first
    out = mlp_forward(D, p, Ud).cpu().numpy()
    assert np.mean(np.sum((out - T) ** 2, axis=1)) < 0.1 * np.mean(np.sum(T ** 2, axis=1))


def test_samples_are_moments_and_exact_pair_terms(torch_cuda):
    """Training rows the library gathers after 3 steps (FP64 path): the RFF
    moments and the exact pair terms at the sampled particles, against the
    oracle's at its own Y*_3 = F_h(X_3); each row's particle is the oracle
    particle nearest to the row's y."""
    from paper_2105_09688_amd.ssm import SSM
    w = _small_w(N=3000)
    N, ens, h = w["systems"][0]
    X = oracle.init_state(w, ens, N)
    for n in range(3):
        X, _ = oracle.step(w, ens, h, n, X)
    _, Y = oracle.step(w, ens, h, 3, X)
    with SSM(w, precision="fp64") as s:
        s.step(3)
        U, T = s.surrogate_samples(500, seed=11)
    U, T = U.cpu().numpy().astype(np.float64), T.cpu().numpy().astype(np.float64)
    om = oracle.rff_omegas(w["seed"], D, 16, w["b"]["ell"])
    mref = oracle.rff_moments(Y, om)
    assert np.max(np.abs(U[:, D:] - mref[None, :])) <= 2e-5
    dist = np.sqrt(((U[:, :D, None] - Y[None, :, :]) ** 2).sum(axis=1))  # [rows, N]
    idx = np.argmin(dist, axis=1)
    two = np.partition(dist, 1, axis=1)
    assert np.max(two[:, 0]) <= 1e-6 and np.min(two[:, 1]) >= 1e-5  # float32 rows, unambiguous match
    Kref = oracle.pair_sum_at(Y, w["b"]["ell"], idx) * w["b"]["g"]
    assert np.max(np.abs(T - Kref.T)) <= 2e-6


@pytest.fixture(scope="module")
def trained_small(torch_cuda):
    """A small network trained on another ensemble, the exact run's X_T and
    its workload (shared by the tests of the surrogate step)."""
    torch = torch_cuda
    from paper_2105_09688_amd.ssm import SSM, mlp_init, mlp_train
    w = _small_w()
    wt = W.with_systems(w, [(4096, 1, 2.0 ** -9)])
    Us, Ts = [], []
    with SSM(wt, precision="fp32_kahan") as s:
        for t in range(8):
            U, T = s.surrogate_samples(4096, seed=t)
            Us.append(U)
            Ts.append(T)
            s.step(4)
    U, T = torch.cat(Us), torch.cat(Ts)
    p = torch.tensor(mlp_init(D, seed=0), device="cuda")
    hist = mlp_train(D, p, U, T, steps=800, batch=1024, lr=2e-3, seed=3)
    _say(f"train loss {hist[0]:.3e} -> {hist[-1]:.3e}")
    # the multi-launch exact path: the one a surrogate context falls back to
    with SSM(w, precision="fp32_kahan", persistent=-1) as ex:
        ex.run()
        X_exact = ex.state(0)
    return w, p.cpu().numpy(), X_exact


def _surrogate_run(w, master, **enable):
    from paper_2105_09688_amd.ssm import SSM
    with SSM(w, precision="fp32_kahan") as s:
        s.surrogate_load(master)
        s.surrogate_enable(**enable)
        s.run()
        return s.state(0), s.info()


def _rms(A, B):
    return float(np.sqrt(np.mean(np.sum((A - B) ** 2, axis=0))))


def test_surrogate_step_and_fallback(trained_small):
    """A surrogate that fails its checks leaves the run identical to the
    exact one; one that is always accepted changes the run only by its own
    error; the counters reflect both."""
    w, master, X_exact = trained_small
    # impossible tolerance: every check fails, every tick is exact
    X_fb, info = _surrogate_run(w, master, check_every=4, tol=1e-12)
    _say(f"fallback run: {info['surr_checks']} checks, last err {info['surr_last_err']:.3e}")
    assert info["surr_ticks"] == 0 and info["surr_checks"] == 8
    assert info["surr_fallback_ticks"] == 32 - 8
    assert np.array_equal(X_fb, X_exact)
    # accepting tolerance: every non-check tick uses the network
    X_s, info = _surrogate_run(w, master, check_every=4, tol=1e9)
    _say(f"surrogate run: {info['surr_ticks']} ticks, max err {info['surr_max_err']:.3e}")
    assert info["surr_ticks"] == 32 - 8 and info["surr_fallback_ticks"] == 0
    assert 0.0 < info["surr_max_err"] < 1.0
    d_rms = _rms(X_s, X_exact)
    _say(f"pathwise rms difference to exact: {d_rms:.3e}")
    assert d_rms < 0.05


def test_surrogate_residual_mode_is_closer_than_gain_mode(trained_small):
    """The residual carried from the last check removes most of the network's
    error: smaller check errors than the bare network, and a run closer to the
    exact one than the gained network's."""
    w, master, X_exact = trained_small
    X_g, info_g = _surrogate_run(w, master, check_every=4, tol=1e9, mode="gain")
    X_r, info_r = _surrogate_run(w, master, check_every=4, tol=1e9, mode="residual")
    d_g, d_r = _rms(X_g, X_exact), _rms(X_r, X_exact)
    _say(f"gain: last err {info_g['surr_last_err']:.3e}, rms {d_g:.3e}; residual: last err "
         f"{info_r['surr_last_err']:.3e} (bare {info_r['surr_last_raw_err']:.3e}), rms {d_r:.3e}")
    assert info_r["surr_ticks"] == 32 - 8 and info_r["surr_checks"] == 8
    assert info_r["surr_gain"] == [1.0] * D
    assert info_r["surr_last_err"] < 0.5 * info_r["surr_last_raw_err"]
    assert d_r < 0.5 * d_g


def test_surrogate_residual_mode_first_check_and_errors(torch_cuda):
    """The first check has no stored residual: its error is the bare
    network's; the mode checks its arguments."""
    from paper_2105_09688_amd import SSMError
    from paper_2105_09688_amd.ssm import SSM, mlp_init
    w = _small_w(N=2048)
    with SSM(w, precision="fp32_kahan") as s:
        s.surrogate_load(mlp_init(D, seed=4))
        with pytest.raises(ValueError):
            s.surrogate_enable(check_every=4, tol=1e-3, mode="residual-typo")
        s.surrogate_enable(check_every=4, tol=1e9, mode="residual")
        s.step(1)
        info = s.info()
    assert info["surr_checks"] == 1
    assert info["surr_last_err"] == info["surr_last_raw_err"] > 0.0
    # every system must step on check ticks
    wb = W.with_systems(w, [(1024, 0, 2.0 ** -9), (1024, 1, 2.0 ** -8)])
    with SSM(wb, precision="fp32_kahan") as s:
        s.surrogate_load(mlp_init(D, seed=4))
        with pytest.raises(SSMError):
            s.surrogate_enable(check_every=3, tol=1e-3, mode="residual")
        s.surrogate_enable(check_every=4, tol=1e-3, mode="residual")


def test_surrogate_residual_mode_zero_network_matches_oracle(torch_cuda):
    """With all weights zero the network outputs 0, so in residual mode the
    pair term between checks is the exact one frozen at the last check (the
    check ticks use the fresh exact term).  The oracle runs the same scheme
    from its exact step: X_{n+1} = step(X_n) + h g (P(Y_{c(n)}) - P(Y_n)) with
    c(n) the last check step; FP32 bar 1e-4."""
    from paper_2105_09688_amd.ssm import SSM, mlp_num_params
    h = 2.0 ** -9
    w = _small_w(N=1536, T=24 * h)
    every = 4
    with SSM(w, precision="fp32_kahan") as s:
        s.surrogate_load(np.zeros(mlp_num_params(D), dtype=np.float32))
        s.surrogate_enable(check_every=every, tol=1e9, mode="residual")
        s.run()
        info = s.info()
        X_gpu = s.state(0)
    assert info["surr_ticks"] == 24 - 24 // every
    _say(f"zero network, residual mode: last err {info['surr_last_err']:.3e}")
    N, ens, _ = w["systems"][0]
    g, ell = w["b"]["g"], w["b"]["ell"]
    X = oracle.init_state(w, ens, N)
    P_frozen = None
    for n in range(24):
        X_next, Y = oracle.step(w, ens, h, n, X)
        P = oracle.pair_sum(Y, ell)
        if n % every == 0:
            P_frozen = P
        X = X_next + h * g * (P_frozen - P)
    err = np.max(np.abs(X_gpu - X) / np.maximum(1.0, np.abs(X)))
    _say(f"max rel err vs oracle emulation {err:.3e}")
    assert err <= 1e-4
    # and the frozen term really differs from the exact run
    X_ex = oracle.run(w)[0]
    assert np.max(np.abs(X - X_ex)) > 1e-6


def test_recheck_with_failing_checks_is_the_exact_run(trained_small):
    """With rechecks on and an impossible tolerance every tick is a check
    (scheduled or recheck), every update uses the exact sums, and the run is
    the exact one bitwise."""
    w, master, X_exact = trained_small
    X_fb, info = _surrogate_run(w, master, check_every=4, tol=1e-12, recheck=True)
    _say(f"recheck fallback run: {info['surr_checks']} checks ({info['surr_rechecks']} rechecks)")
    assert info["surr_checks"] == 32 and info["surr_rechecks"] == 32 - 8
    assert info["surr_ticks"] == 0 and info["surr_fallback_ticks"] == 0
    assert np.array_equal(X_fb, X_exact)
    # an accepting tolerance never falls back, so it never rechecks
    _, info = _surrogate_run(w, master, check_every=4, tol=1e9, recheck=True)
    assert info["surr_rechecks"] == 0 and info["surr_ticks"] == 32 - 8
    # the switch takes 0 or 1 only
    from paper_2105_09688_amd import SSMError, _lib
    from paper_2105_09688_amd.ssm import SSM
    with SSM(w, precision="fp32_kahan") as s:
        with pytest.raises(SSMError):
            _lib.check(_lib.load().ssm_surrogate_recheck(s._h, 2))


def test_recheck_only_where_every_system_steps(torch_cuda):
    """In a context of two step sizes (strides 1 and 2) a recheck falls only
    on ticks where both systems step: with an impossible tolerance, checks on
    every even tick (8 scheduled every 4 ticks, 8 rechecks), the odd ticks
    exact as fallback ticks, and the run bitwise the exact one."""
    from paper_2105_09688_amd.ssm import SSM, mlp_init
    h = 2.0 ** -9
    w = W.with_systems(_small_w(N=1024, T=32 * h), [(1024, 0, h), (1000, 1, 2 * h)])
    with SSM(w, precision="fp32_kahan", persistent=-1) as ex:
        ex.run()
        X_ex = ex.states()
    with SSM(w, precision="fp32_kahan") as s:
        s.surrogate_load(mlp_init(D, seed=4))
        s.surrogate_enable(check_every=4, tol=1e-12, mode="residual", recheck=True)
        s.run()
        info = s.info()
        X = s.states()
    _say(f"two step sizes: {info['surr_checks']} checks ({info['surr_rechecks']} rechecks), "
         f"{info['surr_fallback_ticks']} fallback ticks")
    assert (info["surr_checks"], info["surr_rechecks"], info["surr_fallback_ticks"], info["surr_ticks"]) == (16, 8, 16, 0)
    for a, b in zip(X, X_ex):
        assert np.array_equal(a, b)


def test_recheck_zero_network_matches_oracle(torch_cuda):
    """Residual mode with an all-zero network and rechecks: the prediction
    is the exact term frozen at the last check, so a check's error is the
    relative change of the exact term since that check.  With the tolerance
    between the one-tick and the three-tick change, each scheduled check
    (every 4 ticks, three ticks after the last recheck) fails, the recheck on
    the next tick passes, and the two ticks after it use the frozen term.
    The oracle runs the same rule from its exact step, with its own FP64
    errors deciding (each at least 20 % away from the tolerance); the counts
    must agree and the states meet the FP32 bar 1e-4."""
    from paper_2105_09688_amd.ssm import SSM, mlp_num_params
    h = 2.0 ** -9
    w = _small_w(N=1536, T=24 * h)
    every, tol = 4, 2.4e-2
    with SSM(w, precision="fp32_kahan") as s:
        s.surrogate_load(np.zeros(mlp_num_params(D), dtype=np.float32))
        s.surrogate_enable(check_every=every, tol=tol, mode="residual", recheck=True)
        s.run()
        info = s.info()
        X_gpu = s.state(0)
    N, ens, _ = w["systems"][0]
    g, ell = w["b"]["g"], w["b"]["ell"]
    X = oracle.init_state(w, ens, N)
    P_frozen, fallback, checks, rechecks, net = None, False, 0, 0, 0
    for n in range(24):
        X_next, Y = oracle.step(w, ens, h, n, X)
        P = oracle.pair_sum(Y, ell)
        sched = n % every == 0
        if sched or fallback:
            q = np.zeros_like(P) if P_frozen is None else P_frozen
            err = float(np.sqrt(np.sum((q - P) ** 2) / np.sum(P ** 2)))
            assert abs(err / tol - 1.0) > 0.2, f"tick {n}: error {err:.3e} too close to the tolerance"
            checks += 1
            rechecks += 0 if sched else 1
            fallback = not err <= tol
            P_frozen = P
            X = X_next
        else:
            net += 1
            X = X_next + h * g * (P_frozen - P)
    _say(f"recheck, zero network: {info['surr_checks']} checks ({info['surr_rechecks']} rechecks), "
         f"{info['surr_ticks']} network ticks; oracle {checks} ({rechecks}), {net}")
    assert (info["surr_checks"], info["surr_rechecks"], info["surr_ticks"]) == (checks, rechecks, net)
    assert rechecks > 0 and net > 0
    err = np.max(np.abs(X_gpu - X) / np.maximum(1.0, np.abs(X)))
    _say(f"max rel err vs oracle emulation {err:.3e}")
    assert err <= 1e-4


@pytest.fixture(scope="module")
def rmse_case(torch_cuda):
    """The reduced surrogate case for the strong-error comparisons: d = 2,
    N = 1024, h = 2^-9, T = 1/4; the oracle's exact run and its 2^-13 proxy
    on the same paths (Section 3's strong error), and a network trained on
    exact runs of ensembles 1 and 2 at N = 4096."""
    torch = torch_cuda
    from paper_2105_09688_amd.ssm import SSM, mlp_init, mlp_train
    h, hf = 2.0 ** -9, 2.0 ** -13
    w = W.surrogate_d2(N=1024, h=h, h_fine=hf)
    w["T"] = 0.25
    ref_w = W.with_h(w, hf)
    _say("oracle exact run and 2^-13 proxy")
    o = oracle.run(w)[0]
    o_ref = oracle.run(ref_w)[0]
    Us, Ts = [], []
    for e in (1, 2):
        with SSM(W.with_systems(w, [(4096, e, h)]), precision="fp32_kahan") as s:
            for t in range(32):
                U, T = s.surrogate_samples(4096, seed=100 * e + t)
                Us.append(U)
                Ts.append(T)
                s.step(4)
    p = torch.tensor(mlp_init(D, seed=0), device="cuda")
    mlp_train(D, p, torch.cat(Us), torch.cat(Ts), steps=6000, batch=2048, lr=1e-3, seed=1)
    mlp_train(D, p, torch.cat(Us), torch.cat(Ts), steps=3000, batch=2048, lr=2e-4, seed=2)
    return w, o, o_ref, p.cpu().numpy()


def test_surrogate_run_rmse_within_5_percent_of_oracle(rmse_case):
    """Strong error at h = 2^-9 against a 2^-13 proxy solution on the same
    paths (Section 3), N = 1024, T = 1/4: the surrogate run (residual mode,
    checks every 16 steps, tolerance 1e-2; most ticks on the network) is
    within 5 % of the oracle's exact run.  (At this N the finite-N part of the
    pair term moves by about 5e-3 between checks, so the 1e-3 tolerance of the
    surrogate case falls back on every interval; that tolerance is tested at
    N = 8192 below.)"""
    from paper_2105_09688_amd.ssm import SSM
    w, o, o_ref, master = rmse_case
    r_oracle = oracle.strong_error(o, o_ref)
    with SSM(w, precision="fp32_kahan") as s:
        s.surrogate_load(master)
        s.surrogate_enable(check_every=16, tol=1e-2, mode="residual")
        s.run()
        info = s.info()
        X = s.state(0)
    r_gpu = errstats.strong_error(X, o_ref)
    _say(f"rmse oracle exact {r_oracle:.4e}, gpu surrogate {r_gpu:.4e} (ratio {r_gpu / r_oracle:.4f}); "
         f"surrogate ticks {info['surr_ticks']}, fallback ticks {info['surr_fallback_ticks']}, last / max check err "
         f"{info['surr_last_err']:.3e} / {info['surr_max_err']:.3e}")
    assert info["surr_ticks"] >= 60  # of 120 non-check ticks
    assert abs(r_gpu - r_oracle) <= 0.05 * r_oracle


def _golden(name):
    import json
    import os
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fixed_rmse.json")) as fh:
        return json.load(fh)[name]


@pytest.fixture(scope="module")
def fixed_rmse_case(torch_cuda):
    """The surrogate case's coefficients at N = 8192, T = 1, h = 2^-9 (512
    steps, 32 checks), with the oracle's strong error against a 2^-13 proxy
    stored in tests/golden/fixed_rmse.json (written by the oracle alone).  The
    GPU side takes its proxy from the FP64 path at 2^-13 on the same paths;
    that the GPU FP64 path reproduces the oracle's strong error (to 1e-6
    relative, both runs and the proxy being pathwise within about 1e-10 of
    the oracle's) pins the chain.  The network is trained on exact runs of
    ensembles 1 and 2 at N = 2^14 (32 states each)."""
    torch = torch_cuda
    from paper_2105_09688_amd.ssm import SSM, mlp_init, mlp_train
    g = _golden("surrogate_reduced")
    h, hf, N = g["h"], g["proxy_h"], g["N"]
    w = W.surrogate_d2(N=N, h=h, h_fine=hf)
    assert w["T"] == g["T"]
    with SSM(W.with_h(w, hf), precision="fp64") as r:
        r.run()
        X_ref = r.state(0)
    with SSM(w, precision="fp64") as e64:
        e64.run()
        r64 = errstats.strong_error(e64.state(0), X_ref)
    with SSM(w, precision="fp32_kahan") as ex:
        ex.run()
        X_ex = ex.state(0)
    _say(f"N={N}: oracle strong error {g['rmse']:.6e}, GPU FP64 {r64:.6e}, GPU FP32-compensated "
         f"{errstats.strong_error(X_ex, X_ref):.6e}")
    assert abs(r64 - g["rmse"]) <= 1e-6 * g["rmse"]
    Us, Ts = [], []
    for e in (1, 2):
        with SSM(W.with_systems(w, [(2 ** 14, e, h)]), precision="fp32_kahan") as s:
            for t in range(0, 512, 16):
                U, T = s.surrogate_samples(2 ** 16, seed=1000 * e + t)
                Us.append(U)
                Ts.append(T)
                s.step(16)
    U, T = torch.cat(Us), torch.cat(Ts)
    p = torch.tensor(mlp_init(D, seed=0), device="cuda")
    for steps, lr, seed in ((32000, 1e-3, 1), (16000, 2e-4, 2), (8000, 4e-5, 3)):
        mlp_train(D, p, U, T, steps=steps, batch=4096, lr=lr, seed=seed)
    return w, g["rmse"], X_ref, X_ex, p.cpu().numpy()


def _surr_run(w, weights, tol, every=16):
    from paper_2105_09688_amd.ssm import SSM
    with SSM(w, precision="fp32_kahan") as s:
        s.surrogate_load(weights)
        s.surrogate_enable(check_every=every, tol=tol, mode="residual")
        s.run()
        return s.state(0), s.info()


def test_surrogate_rmse_within_5_percent_of_oracle_at_tolerance_1e3(fixed_rmse_case):
    """The surrogate case's check rule (exact check every 16 steps, fallback
    above 1e-3 relative drift error), residual mode: the strong error at
    h = 2^-9 is within 5 % of the oracle's exact run (Section 3's strong
    error, the metric's "fixed rMSE"), with at least 200 of the 480 non-check
    ticks on the network."""
    w, r_oracle, X_ref, X_ex, master = fixed_rmse_case
    X, info = _surr_run(w, master, 1e-3)
    r_gpu = errstats.strong_error(X, X_ref)
    _say(f"tol 1e-3 at N={w['systems'][0][0]}: rmse oracle {r_oracle:.5e}, surrogate {r_gpu:.5e} (ratio "
         f"{r_gpu / r_oracle:.4f}); surrogate ticks {info['surr_ticks']}, fallback ticks "
         f"{info['surr_fallback_ticks']}, check err last / max {info['surr_last_err']:.3e} / {info['surr_max_err']:.3e}, "
         f"pathwise rms vs exact {_rms(X, X_ex):.3e}")
    assert info["surr_ticks"] >= 200
    assert abs(r_gpu - r_oracle) <= 0.05 * r_oracle


def test_trained_network_gains_over_the_frozen_exact_term(fixed_rmse_case):
    """What the trained network adds over the method without it.  In residual
    mode an all-zero network leaves the exact pair term frozen at the last
    check (the scheme without a network); the trained network adds its
    prediction of the term's change since that check.  Same cadence (16) and
    tolerance (1e-3): the trained network keeps at least 200 ticks on the
    cheap path where the frozen term keeps at most a tenth of that; with every
    check accepted (tolerance 1e9) its check errors are at least 5x smaller,
    its path at least 5x closer to the exact run's, and its strong error
    within 5 % of the oracle's where the frozen term's is not."""
    from paper_2105_09688_amd.ssm import mlp_num_params
    w, r_oracle, X_ref, X_ex, master = fixed_rmse_case
    zeros = np.zeros(mlp_num_params(D), dtype=np.float32)
    res = {}
    for name, weights in (("trained", master), ("frozen", zeros)):
        for tol in (1e-3, 1e9):
            X, info = _surr_run(w, weights, tol)
            r = errstats.strong_error(X, X_ref)
            res[name, tol] = dict(ticks=info["surr_ticks"], last=info["surr_last_err"], max=info["surr_max_err"],
                                  rms=_rms(X, X_ex), ratio=r / r_oracle)
            _say(f"{name} tol {tol:g}: surrogate ticks {info['surr_ticks']}, check err last / max "
                 f"{info['surr_last_err']:.3e} / {info['surr_max_err']:.3e}, pathwise rms vs exact "
                 f"{res[name, tol]['rms']:.3e}, rmse ratio vs oracle {r / r_oracle:.4f}")
    t, f = res["trained", 1e-3], res["frozen", 1e-3]
    assert t["ticks"] >= 200 and f["ticks"] <= 0.1 * t["ticks"]
    t, f = res["trained", 1e9], res["frozen", 1e9]
    assert t["last"] <= 0.2 * f["last"]
    assert t["rms"] <= 0.2 * f["rms"]
    assert abs(t["ratio"] - 1.0) <= 0.05 < abs(f["ratio"] - 1.0)


def test_trained_surrogate_gains_over_the_exact_method(torch_cuda):
    """What the network buys: at d = 2, N = 2^16 (64 steps of h = 2^-9, exact
    check every 16), a network trained on other ensembles runs the step at
    least twice as fast as the exact O(N^2) method, with most ticks on the
    network and the path within 1e-3 (RMS) of the exact one."""
    torch = torch_cuda
    from paper_2105_09688_amd.ssm import SSM, mlp_init, mlp_train
    h = 2.0 ** -9
    w = W.surrogate_d2(N=2 ** 16, h=h, h_fine=h)
    w["T"] = 64 * h
    Us, Ts = [], []
    for e in (1, 2):
        with SSM(W.with_systems(w, [(2 ** 14, e, h)]), precision="fp32_kahan") as s:
            for t in range(16):
                U, T = s.surrogate_samples(4096, seed=300 * e + t)
                Us.append(U)
                Ts.append(T)
                s.step(4)
    p = torch.tensor(mlp_init(D, seed=0), device="cuda")
    mlp_train(D, p, torch.cat(Us), torch.cat(Ts), steps=4000, batch=2048, lr=1e-3, seed=1)
    mlp_train(D, p, torch.cat(Us), torch.cat(Ts), steps=2000, batch=2048, lr=2e-4, seed=2)
    master = p.cpu().numpy()

    def timed(setup=None):
        s = SSM(w, precision="fp32_kahan")
        if setup:
            setup(s)
        s.sync()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        s.run()
        e1.record()
        torch.cuda.synchronize()
        info, X = s.info(), s.state(0)
        s.close()
        return e0.elapsed_time(e1), info, X

    timed()  # warm-up of both paths' kernels
    t_ex, _, X_ex = timed()

    def enable(s):
        s.surrogate_load(master)
        s.surrogate_enable(check_every=16, tol=1e-2, mode="residual")

    timed(enable)
    t_su, info, X_su = timed(enable)
    rms = float(np.sqrt(np.mean(np.sum((X_su - X_ex) ** 2, axis=0))))
    _say(f"exact {t_ex:.2f} ms, surrogate {t_su:.2f} ms ({t_ex / t_su:.1f}x), surrogate ticks "
         f"{info['surr_ticks']}, last check err {info['surr_last_err']:.3e}, rms vs exact {rms:.2e}")
    assert info["surr_ticks"] >= 40  # of 60 non-check ticks
    assert t_ex / t_su >= 2.0
    assert rms < 1e-3


def test_library_training_gives_a_usable_surrogate(torch_cuda):
    """ssm_surrogate_train: exact runs of ensembles 1-2 (N = 4096, rows at 32
    states each), Adam in two phases, loaded into the context; the same
    residual-mode run as above then stays within 5 % of the oracle's exact
    strong error with most ticks on the network.  The fresh weights follow
    the stated law (matrices uniform on +-sqrt(6 / (fan_in + fan_out)), zero
    biases), seen through one Adam step of negligible size."""
    from paper_2105_09688_amd.ssm import SSM
    h, hf = 2.0 ** -9, 2.0 ** -13
    w = W.surrogate_d2(N=1024, h=h, h_fine=hf)
    w["T"] = 0.25
    ref_w = W.with_h(w, hf)
    _say("oracle exact run and 2^-13 proxy")
    o = oracle.run(w)[0]
    o_ref = oracle.run(ref_w)[0]
    r_oracle = oracle.strong_error(o, o_ref)
    rows = 2 * 32 * 4096
    with SSM(w, precision="fp32_kahan") as s:
        _say("fresh weights")
        p0, _ = s.surrogate_train(n_samples=2 * 32 * 64, n_ens=2, ens0=1, N=512, snapshots=32, steps=1,
                                  batch=64, lr=1e-30, seed=9)
        off, in_net = 0, 2 * D + 32
        for (o_, i_) in [(64, in_net), (64, 64), (64, 64), (D, 64)]:
            W_, b_ = p0[off:off + o_ * i_].astype(np.float64), p0[off + o_ * i_:off + o_ * i_ + o_]
            lim = np.sqrt(6.0 / (o_ + i_))
            assert np.max(np.abs(W_)) <= lim * (1 + 1e-6) and np.max(np.abs(b_)) <= 1e-28
            assert abs(W_.mean()) <= 0.2 * lim and abs(W_.var() / (lim * lim / 3.0) - 1.0) <= 0.3
            off += o_ * i_ + o_
        _say("library training")
        p, hist = s.surrogate_train(n_samples=rows, n_ens=2, ens0=1, N=4096, snapshots=32, steps=6000,
                                    batch=2048, lr=1e-3, seed=1)
        assert np.all(np.isfinite(hist)) and np.mean(hist[-50:]) < 0.05 * np.mean(hist[:20])
        p, _ = s.surrogate_train(n_samples=rows, n_ens=2, ens0=1, N=4096, snapshots=32, steps=3000,
                                 batch=2048, lr=2e-4, seed=2, init=p)
        s.surrogate_enable(check_every=16, tol=1e-2, mode="residual")
        s.run()
        info = s.info()
        X = s.state(0)
    r_gpu = errstats.strong_error(X, o_ref)
    _say(f"rmse oracle exact {r_oracle:.4e}, gpu surrogate {r_gpu:.4e}; surrogate ticks {info['surr_ticks']}")
    assert info["surr_ticks"] >= 60
    assert abs(r_gpu - r_oracle) <= 0.05 * r_oracle
