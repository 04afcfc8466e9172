"""Pins of the oracle's learned-surrogate pieces (not in the paper): the MLP
forward pass against torch's float64 modules, its hand-written backward pass
against torch autograd and central finite differences, and the random Fourier
feature moments against closed forms."""
import math

import numpy as np
import pytest

IN, H, OUT = 34, 64, 2


def _params(seed, scale=0.3):
    import oracle
    rng = np.random.default_rng(seed)
    return rng.normal(size=oracle.mlp_num_params(IN, H, OUT)) * scale


def _torch_mlp(p):
    import torch
    sizes = [(H, IN), (H, H), (H, H), (OUT, H)]
    layers, off = [], 0
    for (o, i) in sizes:
        lin = torch.nn.Linear(i, o, dtype=torch.float64)
        with torch.no_grad():
            lin.weight.copy_(torch.tensor(p[off:off + o * i].reshape(o, i)))
            off += o * i
            lin.bias.copy_(torch.tensor(p[off:off + o]))
            off += o
        layers.append(lin)
    seq = torch.nn.Sequential(layers[0], torch.nn.SiLU(), layers[1], torch.nn.SiLU(), layers[2],
                              torch.nn.SiLU(), layers[3])
    return seq


def test_mlp_forward_matches_torch(oracle_mod):
    import torch
    p = _params(1)
    X = np.random.default_rng(2).normal(size=(50, IN))
    got = oracle_mod.mlp_forward(p, X, IN, H, OUT)
    ref = _torch_mlp(p)(torch.tensor(X)).detach().numpy()
    assert np.allclose(got, ref, rtol=1e-13, atol=1e-14)


def test_mlp_gradient_matches_torch_autograd(oracle_mod):
    import torch
    p = _params(3)
    rng = np.random.default_rng(4)
    X = rng.normal(size=(40, IN))
    T = rng.normal(size=(40, OUT))
    loss, g = oracle_mod.mlp_loss_grad(p, X, T, IN, H, OUT)
    net = _torch_mlp(p)
    out = net(torch.tensor(X))
    L = ((out - torch.tensor(T)) ** 2).sum(dim=1).mean()
    L.backward()
    ref = np.concatenate([np.concatenate([m.weight.grad.numpy().ravel(), m.bias.grad.numpy()])
                          for m in net if isinstance(m, torch.nn.Linear)])
    assert loss == pytest.approx(float(L), rel=1e-13)
    assert np.allclose(g, ref, rtol=1e-11, atol=1e-14)


def test_mlp_gradient_matches_central_differences(oracle_mod):
    p = _params(5)
    rng = np.random.default_rng(6)
    X = rng.normal(size=(8, IN))
    T = rng.normal(size=(8, OUT))
    _, g = oracle_mod.mlp_loss_grad(p, X, T, IN, H, OUT)
    idx = rng.choice(p.size, 60, replace=False)
    idx = np.concatenate([idx, [0, IN * H - 1, p.size - 1, p.size - 3]])
    for q in idx:
        eps = 1e-5 * max(1.0, abs(p[q]))
        pp, pm = p.copy(), p.copy()
        pp[q] += eps
        pm[q] -= eps
        fd = (oracle_mod.mlp_loss_grad(pp, X, T, IN, H, OUT)[0] - oracle_mod.mlp_loss_grad(pm, X, T, IN, H, OUT)[0]) / (2 * eps)
        assert abs(fd - g[q]) <= 1e-6 * max(1e-3, abs(g[q])) + 1e-9, (q, fd, g[q])


def test_rff_frequencies_are_gaussian_with_scale_one_over_ell(oracle_mod):
    om = oracle_mod.rff_omegas(0, 2, 4000, 0.5)
    assert abs(om.mean()) < 4 * 2.0 / math.sqrt(om.size)
    assert abs(om.std() - 2.0) < 0.05
    assert np.array_equal(oracle_mod.rff_omegas(0, 2, 16, 1.0), oracle_mod.rff_omegas(0, 2, 40, 1.0)[:16])


def test_rff_moments_closed_forms(oracle_mod):
    om = oracle_mod.rff_omegas(0, 2, 16, 1.0)
    # symmetric two-point cloud {a, -a}: C_k = cos(omega.a), S_k = 0
    a = np.array([0.7, -1.3])
    Y = np.stack([a, -a], axis=1)
    m = oracle_mod.rff_moments(Y, om)
    assert np.allclose(m[:16], np.cos(om @ a), rtol=0, atol=1e-15)
    assert np.allclose(m[16:], 0.0, atol=1e-16)
    # Gaussian cloud N(mu, s^2 I): E cos(w.y) = cos(w.mu) exp(-s^2|w|^2/2), E sin = sin(w.mu) exp(...)
    rng = np.random.default_rng(9)
    mu, s, N = np.array([0.4, -0.2]), 0.6, 200000
    Y = (mu[:, None] + s * rng.normal(size=(2, N)))
    m = oracle_mod.rff_moments(Y, om)
    damp = np.exp(-0.5 * s * s * np.sum(om * om, axis=1))
    assert np.allclose(m[:16], np.cos(om @ mu) * damp, atol=5 / math.sqrt(N))
    assert np.allclose(m[16:], np.sin(om @ mu) * damp, atol=5 / math.sqrt(N))
