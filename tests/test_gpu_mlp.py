"""Parity of the surrogate's HIP kernels (through the C-ABI) with the FP64
oracle run in BF16-emulation mode (operands of every matrix product rounded
to BF16 where the GPU rounds them).

Bounds: the GPU accumulates in FP32 and evaluates GELU in FP32, so a hidden
activation can round to the neighbouring BF16 value (2^-8 relative) where the
oracle does not; the outputs are compared to 2e-3 of their scale and the
gradients to 2e-3 in relative 2-norm (measured differences are far smaller).
"""
import numpy as np
import pytest
import torch

from oracle import mlp as om
from workloads import make_workload, mlp_init, mlp_order

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1312_4746_amd import Context
    c = Context(0)
    yield c
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _net(ctx, n_in, n_out, seed=1):
    from paper_1312_4746_amd import Mlp
    p0 = mlp_init(n_in, 128, n_out, seed)
    return Mlp(ctx, n_in, n_out, dev(p0)), p0.astype(np.float64)


@pytest.mark.parametrize("n_in,n_out,n", [(103, 10, 100), (7, 3, 16), (128, 16, 33), (20, 1, 1)])
def test_forward_matches_oracle(ctx, n_in, n_out, n):
    net, p0 = _net(ctx, n_in, n_out)
    X = np.random.default_rng(2).standard_normal((n, n_in)).astype(np.float32)
    y = net.forward(dev(X)).cpu().numpy().astype(np.float64)
    ref = om.forward(p0, om.Shapes(n_in, 128, n_out), X, emulate_bf16=True)["y"]
    scale = max(1.0, float(np.abs(ref).max()))
    assert np.max(np.abs(y - ref)) <= 2e-3 * scale, float(np.max(np.abs(y - ref)))
    net.close()


def test_params_roundtrip(ctx):
    net, p0 = _net(ctx, 30, 4)
    assert np.array_equal(net.params().cpu().numpy(), p0.astype(np.float32))
    net.close()


@pytest.mark.parametrize("n", [16, 512, 4096])
def test_gradient_matches_oracle(ctx, n):
    n_in, n_out = 103, 10
    net, p0 = _net(ctx, n_in, n_out, seed=3)
    rng = np.random.default_rng(4)
    X = rng.standard_normal((n, n_in)).astype(np.float32) * 0.5
    ell = (rng.standard_normal((n, n_out)) * 5 - 10).astype(np.float32)
    ell[::7, 3] = -80.0  # clipped targets
    g, loss = net.grad(dev(X), dev(ell))
    g = g.cpu().numpy().astype(np.float64)
    T = om.clip_targets(ell.astype(np.float64))
    loss_ref, g_ref = om.loss_and_grad(p0, om.Shapes(n_in, 128, n_out), X, T, emulate_bf16=True)
    rel = np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref)
    assert rel <= 2e-3, rel
    assert abs(float(loss.cpu()) - loss_ref) <= 1e-4 * loss_ref
    # every parameter block is compared (a dropped block fails the norm test above,
    # but check each one separately too)
    sh = om.Shapes(n_in, 128, n_out)
    gb, rb = om.unpack(g, sh), om.unpack(g_ref, sh)
    for name in gb:
        assert np.linalg.norm(gb[name] - rb[name]) <= 5e-3 * np.linalg.norm(rb[name]) + 1e-9, name
    net.close()


def test_training_steps_track_oracle(ctx):
    n_in, n_out, B, steps = 23, 5, 256, 8
    net, p0 = _net(ctx, n_in, n_out, seed=5)
    rng = np.random.default_rng(6)
    X = rng.standard_normal((1000, n_in)).astype(np.float32)
    ell = (np.tanh(X[:, :n_out]) * 3 - 5).astype(np.float32)
    order = mlp_order(1000, steps, B, seed=7)
    trace = net.train(dev(X), dev(ell), dev(order.ravel()), B, lr=1e-3).cpu().numpy()
    p_ref, loss_ref = om.train(p0, om.Shapes(n_in, 128, n_out), X, om.clip_targets(ell), order, lr=1e-3,
                               emulate_bf16=True)
    np.testing.assert_allclose(trace, loss_ref, rtol=2e-3)
    p = net.params().cpu().numpy().astype(np.float64)
    # each Adam step moves a parameter by at most ~lr; the trajectories agree to a
    # small fraction of the total movement
    moved = np.linalg.norm(p_ref - p0)
    assert np.linalg.norm(p - p_ref) <= 0.05 * moved, (np.linalg.norm(p - p_ref), moved)
    net.close()


def test_infer_equals_forward_on_features(ctx):
    from paper_1312_4746_amd import mlp_features
    w = make_workload("mlp_small", H=37, W=53, R=3, p=5, k=40, seed=9, per_region=5)
    rgb = dev(w.rgb)
    alpha = ctx.analyze_patches(rgb, w.p, w.mask_sigma, dev(w.omega))
    net, _ = _net(ctx, 5 + w.k, w.L, seed=10)
    y_all = net.infer(rgb, alpha)
    pix = torch.arange(w.N, dtype=torch.int32, device="cuda")
    X = mlp_features(ctx, rgb, alpha, pix)
    y_x = net.forward(X)
    assert torch.equal(y_all, y_x)
    ref = om.features(w.rgb, alpha.cpu().numpy(), np.arange(w.N))
    np.testing.assert_allclose(X.cpu().numpy(), ref, rtol=1e-7, atol=0)
    net.close()


def test_errors(ctx):
    from paper_1312_4746_amd import CosparseError, Mlp
    from paper_1312_4746_amd.binding import param_count
    assert param_count(103, 64, 10) == 0
    assert param_count(129, 128, 10) == 0
    assert param_count(103, 128, 17) == 0
    with pytest.raises(CosparseError):
        Mlp(ctx, 103, 10, dev(np.zeros(10, np.float32)).new_zeros(31114), hidden=64)
    net, _ = _net(ctx, 8, 2)
    with pytest.raises(CosparseError):
        net.grad(dev(np.zeros((15, 8), np.float32)), dev(np.zeros((15, 2), np.float32)))
    with pytest.raises(CosparseError):
        net.train(dev(np.zeros((32, 8), np.float32)), dev(np.zeros((32, 2), np.float32)),
                  dev(np.zeros(24, np.int32)), 24)
    net.close()


def test_output_bias_is_mean_clipped_target(ctx):
    net, p0 = _net(ctx, 12, 6, seed=12)
    rng = np.random.default_rng(13)
    ell = (rng.standard_normal((777, 6)) * 10 - 20).astype(np.float32)
    net.fit_output_bias(dev(ell))
    p = net.params().cpu().numpy().astype(np.float64)
    sh = om.Shapes(12, 128, 6)
    ref = om.clip_targets(ell.astype(np.float64)).mean(0)
    np.testing.assert_allclose(om.unpack(p, sh)["b3"], ref, rtol=1e-6)
    # the other parameters are untouched
    assert np.array_equal(om.unpack(p, sh)["W3"], om.unpack(p0, sh)["W3"].astype(np.float32))
    net.close()
