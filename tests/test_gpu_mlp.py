"""Parity of the surrogate's HIP kernels (through the C-ABI) with the FP64
oracle run in BF16-emulation mode (operands of every matrix product rounded
to BF16 where the GPU rounds them).

Bounds: the GPU accumulates in FP32 and evaluates GELU in FP32, so a hidden
activation can round to the neighbouring BF16 value where the oracle does
not; the outputs are compared to 2e-3 of their scale.  Gradients are compared
element by element against a first-order bound of those effects
(`grad_error_bound`), and in relative 2-norm.
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


U_F32 = 2.0 ** -24
GELU1_MAX = 1.13     # max |GELU'(z)| = Phi(sqrt 2) + sqrt 2 phi(sqrt 2) = 1.1289
GELU2_MAX = 0.80     # max |GELU''(z)| = 2 phi(0) = 0.7979
# the kernels evaluate erf with Abramowitz-Stegun 7.1.26 (|error| <= 1.5e-7) in
# FP32: GELU(z) is within 0.75e-7 |z| plus a few FP32 roundings, GELU'(z)
# within about 2e-7
GELU_REL_Z = 1e-7
GELU1_ABS = 2e-7


def bf16_discrepancy(v, dv):
    """Bound on |r(v') - r(v)| over |v' - v| <= dv, r the BF16 rounding (the
    GPU rounds its FP32 value v', the oracle its FP64 value v via FP32): dv
    itself, plus a flip to the neighbouring BF16 value where v lies within dv
    (and an FP32 rounding) of a rounding midpoint; a flip moves the result by
    one BF16 ulp, counted as two to cover a binade crossing."""
    a = np.abs(v)
    e = np.floor(np.log2(np.where(a > 0, a, 1.0)))
    ulp = np.ldexp(1.0, (e - 7).astype(int))
    frac = a / ulp - np.floor(a / ulp)
    near = np.abs(frac - 0.5) * ulp <= dv + 2 * U_F32 * a
    return dv + np.where(near & (a > 0), 2 * ulp, 0.0)


def grad_error_bound(flat, sh, X, T):
    """First-order bound on |g_gpu - g_oracle| for every parameter, the oracle
    in BF16-emulation mode.  Sources: FP32 accumulation of every product (n
    terms: n 2^-24 times the sum of the magnitudes), FP32 GELU/GELU' (absolute
    error GELU_REL_Z |z| plus FP32 roundings for GELU, GELU1_ABS for GELU'),
    and the BF16 rounding points, where the GPU's and the oracle's values
    differ by the propagated bound and may round to neighbouring BF16 values
    (bf16_discrepancy).  The discrepancies are propagated through the absolute
    values of the weights and of the GELU derivatives (bounded by GELU1_MAX,
    and their change by GELU2_MAX times the change of z), then doubled to
    cover second-order terms."""
    q = om.round_bf16
    p = om.unpack(flat, sh)
    f = om.forward(flat, sh, X, emulate_bf16=True)
    B, L = f["y"].shape
    aX = np.abs(q(f["X"]))
    W1, W2, W3 = (np.abs(q(p[k])) for k in ("W1", "W2", "W3"))
    # forward
    dz1 = sh.n_in * U_F32 * (aX @ W1.T + np.abs(p["b1"]))
    dh1 = GELU1_MAX * dz1 + GELU_REL_Z * np.abs(f["z1"]) + 4 * U_F32 * np.abs(f["h1"])
    qh1 = np.abs(q(f["h1"]))
    dqh1 = bf16_discrepancy(f["h1"], dh1)
    dz2 = dqh1 @ W2.T + sh.hidden * U_F32 * (qh1 @ W2.T + np.abs(p["b2"]))
    dh2 = GELU1_MAX * dz2 + GELU_REL_Z * np.abs(f["z2"]) + 4 * U_F32 * np.abs(f["h2"])
    qh2 = np.abs(q(f["h2"]))
    dqh2 = bf16_discrepancy(f["h2"], dh2)
    dy_out = dqh2 @ W3.T + sh.hidden * U_F32 * (qh2 @ W3.T + np.abs(p["b3"]))
    # backward
    d = f["y"] - T
    dy = 2.0 * d / (B * L)
    ddy = 2.0 * dy_out / (B * L) + 4 * U_F32 * np.abs(dy)
    qdy = np.abs(q(dy))
    dqdy = bf16_discrepancy(dy, ddy)
    g2 = om.gelu_grad(f["z2"])
    dh2b = q(dy) @ q(p["W3"])
    ddh2 = dqdy @ W3 + sh.n_out * U_F32 * (qdy @ W3)
    dz2b = dh2b * g2
    ddz2 = ddh2 * np.abs(g2) + np.abs(dh2b) * (GELU2_MAX * dz2 + GELU1_ABS) + 2 * U_F32 * np.abs(dz2b)
    qdz2 = np.abs(q(dz2b))
    dqdz2 = bf16_discrepancy(dz2b, ddz2)
    g1 = om.gelu_grad(f["z1"])
    dh1b = q(dz2b) @ q(p["W2"])
    ddh1 = dqdz2 @ W2 + sh.hidden * U_F32 * (qdz2 @ W2)
    dz1b = dh1b * g1
    ddz1 = ddh1 * np.abs(g1) + np.abs(dh1b) * (GELU2_MAX * dz1 + GELU1_ABS) + 2 * U_F32 * np.abs(dz1b)
    qdz1 = np.abs(q(dz1b))
    dqdz1 = bf16_discrepancy(dz1b, ddz1)
    gb = {
        "W3": dqdy.T @ qh2 + qdy.T @ dqh2 + B * U_F32 * (qdy.T @ qh2),
        "b3": ddy.sum(0) + B * U_F32 * np.abs(dy).sum(0),
        "W2": dqdz2.T @ qh1 + qdz2.T @ dqh1 + B * U_F32 * (qdz2.T @ qh1),
        "b2": ddz2.sum(0) + B * U_F32 * np.abs(dz2b).sum(0),
        "W1": dqdz1.T @ aX + B * U_F32 * (qdz1.T @ aX),
        "b1": ddz1.sum(0) + B * U_F32 * np.abs(dz1b).sum(0),
    }
    return 2.0 * om.pack(gb, sh) + 1e-12


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
    # element by element, inside the first-order bound of the rounding effects
    bound = grad_error_bound(p0, om.Shapes(n_in, 128, n_out), X.astype(np.float64), T)
    ratio = np.abs(g - g_ref) / bound
    print(f"n={n}: max |dg|/bound = {ratio.max():.3g}, median {np.median(ratio):.3g}, "
          f"median bound/|g| = {np.median(bound / (np.abs(g_ref) + 1e-30)):.3g}", flush=True)
    assert np.all(ratio <= 1.0), (float(ratio.max()), int(np.argmax(ratio)))
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


def test_surrogate_gain_on_the_2048_workload(ctx):
    """What the trained network gains over the method without it, per image
    and fit included: the surrogate path (BF16 analysis as features, exact
    targets at 2 % of the pixels, 1000 Adam steps, inference with the exact
    data term for pixels whose two best labels are within 2 nats) flips at most
    0.5 % of the label decisions of the exact FP32 data term, takes less time
    than it, and flips fewer labels than the exact data term restricted to a
    random sample subset sized to the surrogate path's whole time."""
    import time

    from paper_1312_4746_amd import LoglikParams, Mlp, mlp_features
    from paper_1312_4746_amd import surrogate as sg
    from workloads import make_config
    w = make_config(4)
    rgb, om = dev(w.rgb), dev(w.omega)
    spix, slab, tpix = dev(w.sample_pix), dev(w.sample_label), dev(w.train_pix)
    prm = LoglikParams(alpha_rho=w.alpha_rho, sigma_c=w.sigma_c, beta_scale=w.beta_scale,
                       rho_floor_px=w.rho_floor_px, colour_levels=w.colour_levels)
    steps, batch = 1000, 4096
    order = dev(mlp_order(len(w.train_pix), steps, batch, seed=w.seed + 101).ravel())
    init = dev(mlp_init(5 + w.k, 128, w.L, seed=w.seed + 100))

    def exact_path():
        _, m, _ = ctx.cosupport_median(rgb, w.p, w.mask_sigma, om, 0.1)
        return m, ctx.label_loglik(rgb, m, w.k, spix, slab, w.L, prm)

    def surrogate_path():
        a, m, _ = ctx.cosupport_median(rgb, w.p, w.mask_sigma, om, 0.1, precision="bf16")
        ell = ctx.label_loglik(rgb, m, w.k, spix, slab, w.L, prm, pix_subset=tpix)
        x = mlp_features(ctx, rgb, a, tpix)
        net = Mlp(ctx, 5 + w.k, w.L, init)
        net.fit_output_bias(ell)
        net.train(x, ell, order, batch, 3e-3)
        y, n = net.infer_fallback(rgb, a, m, w.k, spix, slab, prm, margin=2.0)
        net.close()
        return y, n

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0, r

    exact_path()
    surrogate_path()  # warm-ups (workspace, code objects)
    t_exact, (m32, ll) = timed(exact_path)
    t_sur, (y, n_exact) = timed(surrogate_path)
    q = sg.compare_to_exact(y, ll)
    print(f"surrogate: {q['flip_rate']:.5f} flips, {n_exact} pixels exact, {t_sur * 1e3:.1f} ms per image "
          f"against {t_exact * 1e3:.1f} ms exact", flush=True)
    assert q["flip_rate"] <= 0.005
    assert t_sur < t_exact
    # the method without the network at the surrogate path's time
    t_front, _ = timed(lambda: ctx.cosupport_median(rgb, w.p, w.mask_sigma, om, 0.1))
    frac = max(0.0, (t_sur - t_front) / (t_exact - t_front))
    gen = torch.Generator().manual_seed(w.seed + 102)
    sp2, sl2 = sg.equal_time_subset(spix, slab, w.L, max(w.L, int(w.M * frac)), gen)
    ll2 = ctx.label_loglik(rgb, m32, w.k, sp2, sl2, w.L, prm)
    q2 = sg.compare_to_exact(ll2, ll)
    print(f"equal time: {sp2.numel()} samples ({frac:.2f} of them), {q2['flip_rate']:.5f} flips", flush=True)
    assert q["flip_rate"] < q2["flip_rate"]
