"""Pins of the surrogate oracle (oracle/mlp.py) against independent routes:
the normal CDF of scipy, torch's float64 autograd and Adam, torch's BF16
conversion, central finite differences and closed forms."""
import math

import numpy as np
import pytest
import torch
from scipy.stats import norm

from oracle import mlp as om
from workloads import mlp_init, mlp_order


def _tiny(seed=0, n_in=7, n_out=3, B=6):
    rng = np.random.default_rng(seed)
    sh = om.Shapes(n_in, 5, n_out)
    flat = rng.standard_normal(sh.count) * 0.5
    X = rng.standard_normal((B, n_in))
    T = rng.standard_normal((B, n_out))
    return sh, flat, X, T


def _torch_net(flat, sh, X, T):
    p = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in om.unpack(flat, sh).items()}
    x = torch.tensor(X, dtype=torch.float64)
    h1 = torch.nn.functional.gelu(torch.nn.functional.linear(x, p["W1"], p["b1"]), approximate="none")
    h2 = torch.nn.functional.gelu(torch.nn.functional.linear(h1, p["W2"], p["b2"]), approximate="none")
    y = torch.nn.functional.linear(h2, p["W3"], p["b3"])
    loss = torch.nn.functional.mse_loss(y, torch.tensor(T, dtype=torch.float64))
    loss.backward()
    g = np.concatenate([p[name].grad.numpy().ravel() for name, _ in sh.sizes])
    return y.detach().numpy(), float(loss.detach()), g


def test_gelu_is_z_times_normal_cdf():
    z = np.linspace(-8, 8, 1001)
    np.testing.assert_allclose(om.gelu(z), z * norm.cdf(z), rtol=1e-13, atol=1e-15)
    assert om.gelu(np.array([0.0]))[0] == 0.0
    # Phi(1) = 0.841344746068542948...
    assert abs(om.gelu(np.array([1.0]))[0] - 0.8413447460685429) < 1e-15


def test_gelu_grad_central_differences():
    z = np.linspace(-6, 6, 241)
    h = 1e-6
    fd = (om.gelu(z + h) - om.gelu(z - h)) / (2 * h)
    np.testing.assert_allclose(om.gelu_grad(z), fd, atol=1e-8)


def test_forward_and_gradient_match_torch_float64():
    sh, flat, X, T = _tiny()
    y_t, loss_t, g_t = _torch_net(flat, sh, X, T)
    f = om.forward(flat, sh, X)
    np.testing.assert_allclose(f["y"], y_t, rtol=1e-12, atol=1e-12)
    loss, g = om.loss_and_grad(flat, sh, X, T)
    assert abs(loss - loss_t) <= 1e-12 * max(1.0, abs(loss_t))
    np.testing.assert_allclose(g, g_t, rtol=1e-10, atol=1e-13)


def test_gradient_central_finite_differences():
    sh, flat, X, T = _tiny(seed=3)
    _, g = om.loss_and_grad(flat, sh, X, T)
    h = 1e-6
    idx = np.random.default_rng(1).choice(sh.count, size=40, replace=False)
    for i in idx:
        e = np.zeros_like(flat)
        e[i] = h
        lp, _ = om.loss_and_grad(flat + e, sh, X, T)
        lm, _ = om.loss_and_grad(flat - e, sh, X, T)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(abs(g[i]), 1e-2), (i, fd, g[i])


def test_adam_first_step_closed_form():
    """After one step m_hat = g and v_hat = g^2, so every parameter moves by
    lr * g / (|g| + eps)."""
    g = np.array([3.0, -2e-3, 0.5, -7.0])
    w0 = np.array([1.0, 2.0, -1.0, 0.0])
    w, m, v = om.adam_step(w0, g, np.zeros(4), np.zeros(4), 1, 1e-3)
    np.testing.assert_allclose(w, w0 - 1e-3 * g / (np.abs(g) + om.ADAM_EPS), rtol=0, atol=1e-15)


def test_adam_matches_torch_optim():
    rng = np.random.default_rng(4)
    w = rng.standard_normal(12)
    grads = rng.standard_normal((6, 12))
    pt = torch.tensor(w.copy(), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([pt], lr=2e-3, betas=(0.9, 0.999), eps=1e-8)
    m = np.zeros(12)
    v = np.zeros(12)
    for t in range(6):
        pt.grad = torch.tensor(grads[t], dtype=torch.float64)
        opt.step()
        w, m, v = om.adam_step(w, grads[t], m, v, t + 1, 2e-3)
    np.testing.assert_allclose(w, pt.detach().numpy(), rtol=1e-13, atol=1e-15)


def test_round_bf16_matches_torch():
    rng = np.random.default_rng(5)
    x = np.concatenate([rng.standard_normal(2000) * 10.0 ** rng.integers(-6, 6, 2000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.0078125, 1.005859375, 3.0e38, -1e-40]])
    ref = torch.tensor(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    got = om.round_bf16(x)
    assert np.array_equal(got, ref)


def test_clip_targets():
    ell = np.array([[-1.0, -30.0, -21.0, -20.5], [5.0, 5.0, -100.0, 4.0]])
    t = om.clip_targets(ell)
    np.testing.assert_array_equal(t, [[-1.0, -21.0, -21.0, -20.5], [5.0, 5.0, -15.0, 4.0]])
    assert np.all(t >= ell)


def test_emulated_forward_is_close_to_exact():
    sh, flat, X, T = _tiny(seed=6)
    a = om.forward(flat, sh, X)["y"]
    b = om.forward(flat, sh, X, emulate_bf16=True)["y"]
    assert np.max(np.abs(a - b)) < 0.05 * np.max(np.abs(a)) and not np.array_equal(a, b)


def test_training_reduces_loss():
    rng = np.random.default_rng(7)
    sh = om.Shapes(4, 16, 2)
    X = rng.standard_normal((256, 4))
    T = np.stack([np.sin(X[:, 0]) + X[:, 1], X[:, 2] * X[:, 3]], 1)
    flat0 = mlp_init(4, 16, 2, seed=11).astype(np.float64)
    order = mlp_order(256, 120, 32, seed=12)
    _, losses = om.train(flat0, sh, X, T, order, lr=1e-2)
    assert losses[-10:].mean() < 0.3 * losses[:10].mean()


def test_features_layout():
    rng = np.random.default_rng(8)
    H, W, k = 5, 7, 3
    rgb = rng.random((3, H, W)).astype(np.float32)
    alpha = rng.standard_normal((H * W, k)).astype(np.float32)
    pix = np.array([0, 6, 34, 17])
    x = om.features(rgb, alpha, pix)
    r, c = pix // W, pix % W
    np.testing.assert_array_equal(x[:, :3], rgb.reshape(3, -1)[:, pix].T.astype(np.float64))
    np.testing.assert_allclose(x[:, 3], c / (W - 1))
    np.testing.assert_allclose(x[:, 4], r / (H - 1))
    np.testing.assert_array_equal(x[:, 5:], alpha[pix].astype(np.float64))
    assert x[2, 3] == 1.0 and x[2, 4] == 1.0 and x[0, 3] == 0.0


def test_param_count_of_the_reference_shape():
    assert om.Shapes(103, 128, 10).count == 31114
    assert mlp_init(103, 128, 10, 0).size == 31114
