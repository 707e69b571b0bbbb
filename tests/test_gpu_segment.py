"""Parity of the segmentation kernels (through the C-ABI) with the FP64 oracle
of the convex relaxation (Sec. 3.2, Sec. 4).

Bars.  The FP64 form of the iteration follows the oracle's operation order
without contracted products, so its relaxed solution (returned in FP32) and
energies match the oracle's to the rounding of the output and of a few
reductions (edge metric mean, label-cost sums): |du| <= 2^-24 + 1e-12,
energies within 1e-9 relative.  The FP32 form rounds every step: each
iteration is a nonexpansive map of the previous state plus at most a few
FP32 roundings of quantities bounded by 1 + tau_u |f| + tau_u |div xi|, so its
error grows at most linearly in the iteration count:
|du| <= 32 t 2^-24 (1 + tau_u max|f|), the same relative bound on the
energies.  Labels agree wherever the oracle's two largest u differ by more
than twice the u bound, and elsewhere the GPU's label is one of the oracle's
top labels within that bound.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import segment as osg
from workloads import make_config, make_workload

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.fixture(scope="module")
def ctx():
    from paper_1312_4746_amd import Context
    c = Context(0)
    yield c
    c.close()


def _run(ctx, rgb, ll, lam, nu, iters, prec, gamma=0.0):
    from paper_1312_4746_amd import SegmentParams
    H, W = rgb.shape[1:]
    prm = SegmentParams(lam=lam, gamma=gamma, nu=nu, iterations=iters, precision=prec)
    lab, u, st = ctx.segment(dev(rgb), dev(ll.astype(np.float32)), prm, want_u=True)
    return lab.cpu().numpy().reshape(H, W), u.cpu().numpy(), st


def _oracle(rgb, ll, lam, nu, iters, gamma=0.0):
    H, W = rgb.shape[1:]
    # the oracle reads the same FP32 log-likelihoods
    f = osg.data_term(ll.astype(np.float32).astype(np.float64), H, W)
    g, gm = osg.edge_weight(rgb, gamma)
    return osg.solve(f, g, lam=lam, nu=nu, iterations=iters), f, gm


def _check(ctx, rgb, ll, lam, nu, iters, prec):
    H, W = rgb.shape[1:]
    L = ll.shape[1]
    lab, u, st = _run(ctx, rgb, ll, lam, nu, iters, prec)
    ref, f, gm = _oracle(rgb, ll, lam, nu, iters)
    u_ref = ref["u"].reshape(L, -1).T
    t_u = 0.2 if nu > 0 else 0.25
    if prec == "fp64":
        tol_u, tol_e = 2.0 ** -24 + 1e-12, 1e-9
    else:
        tol_u = 32 * max(iters, 1) * 2.0 ** -24 * (1 + t_u * np.abs(f).max())
        tol_e = tol_u
    du = np.abs(u.astype(np.float64) - u_ref)
    print(f"segment {prec} L={L} t={iters}: max|du| {du.max():.3g} (bound {tol_u:.3g}), energies "
          f"{st['primal']:.9g}/{ref['primal']:.9g} {st['dual']:.9g}/{ref['dual']:.9g}", flush=True)
    assert du.max() <= tol_u, (du.max(), tol_u)
    assert abs(st["gamma"] - gm) <= 1e-12 * gm
    for key in ("primal", "binary", "dual"):
        assert abs(st[key] - ref[key]) <= tol_e * max(1.0, abs(ref[key])), (key, st[key], ref[key])
    # labels: equal where the oracle's decision is clear, a tied top label elsewhere
    srt = np.sort(u_ref, axis=1)
    clear = (srt[:, -1] - srt[:, -2]) > 2 * tol_u if L > 1 else np.ones(u_ref.shape[0], bool)
    ol = ref["labels"].ravel()
    gl = lab.ravel()
    assert np.array_equal(gl[clear], ol[clear])
    top = u_ref[np.arange(u_ref.shape[0]), gl]
    assert np.all(top[~clear] >= srt[~clear, -1] - 2 * tol_u)
    assert st["labels_used"] == len(np.unique(gl))
    return st, ref


def _synthetic_term(w, scale=3.0, seed=0):
    """A data term shaped like a segmentation problem: each region's label is
    favoured, plus noise (random numbers of the test, not of the method)."""
    rng = np.random.default_rng(seed)
    onehot = (w.region.ravel()[:, None] == np.arange(w.L)[None]).astype(np.float64)
    return (scale * onehot + rng.normal(0, scale, (w.N, w.L)) - 5.0).astype(np.float32)


def test_two_iterations_worked_by_hand(ctx):
    """tests/golden/primal_dual_1x2.txt: dyadic values, exact in both precisions
    (g = 1 through gamma = 1/2 on a constant image)."""
    import os
    rows = np.loadtxt(os.path.join(os.path.dirname(__file__), "golden", "primal_dual_1x2.txt"), comments="#")
    rgb = np.zeros((3, 1, 2), np.float32)
    ll = -np.array([[0.0, 1.0], [2.0, 0.0]], np.float32)  # f_0 = (0, 2), f_1 = (1, 0)
    for lam, *u2 in rows:
        for prec in ("fp32", "fp64"):
            _, u, st = _run(ctx, rgb, ll, lam, 0.0, 2, prec, gamma=0.5)
            assert np.array_equal(u.T.ravel(), np.array(u2, np.float32)), (prec, lam, u)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("iters", [0, 1, 3, 60])
def test_tiny_workload(ctx, prec, iters):
    w = make_config(0)
    masks, _, _ = oracle.full_masks(w)
    ll = oracle.label_loglik(w.rgb, masks, w.k, w.sample_pix, w.sample_label, w.L)
    _check(ctx, w.rgb, ll, 1.0, 0.0, iters, prec)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("case", [dict(H=37, W=70, R=4, L=4, nu=0.0, lam=2.0),
                                  dict(H=31, W=33, R=3, L=3, nu=5.0, lam=1.0),
                                  dict(H=1, W=50, R=2, L=2, nu=0.0, lam=1.0),
                                  dict(H=40, W=1, R=2, L=2, nu=0.0, lam=1.0),
                                  dict(H=23, W=29, R=5, L=17, nu=0.0, lam=0.5),
                                  dict(H=20, W=24, R=2, L=1, nu=0.0, lam=1.0)],
                         ids=["L4", "L3_mdl", "row", "column", "L17", "L1"])
def test_small_cases(ctx, prec, case):
    c = dict(case)
    L, nu, lam = c.pop("L"), c.pop("nu"), c.pop("lam")
    w = make_workload("seg", p=3, k=8, seed=11, per_region=3, **c)
    w.L = L
    w.region = w.region % L
    ll = _synthetic_term(w)
    _check(ctx, w.rgb, ll, lam, nu, 40, prec)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_bsds_shape(ctx, prec):
    """481 x 321, 10 labels, 100 iterations, in the launch configuration the
    benchmark times."""
    w = make_config(1)
    ll = _synthetic_term(w, seed=3)
    _check(ctx, w.rgb, ll, 1.0, 0.0, 100, prec)


@pytest.mark.parametrize("prec,nu,L", [("fp64", 0.0, 4), ("fp32", 0.0, 4), ("fp32", 40.0, 3), ("fp32", 0.0, 20)],
                         ids=["fp64", "fp32", "fp32_mdl", "fp32_L20"])
def test_one_launch_form_on_a_large_image(ctx, prec, nu, L):
    """Images of at least 524 288 pixels (eight waves per SIMD with one thread
    per pixel) take the one-launch iteration; smaller ones the two-launch form
    (every other case here).  768 x 704 pixels, 12 iterations (5 with 20
    labels, the kernel that parks its candidates in memory)."""
    w = make_workload("seg_large", H=704, W=768, R=6, p=3, k=8, seed=13, per_region=1)
    w.L = L
    w.region = w.region % L
    ll = _synthetic_term(w, seed=4)
    _check(ctx, w.rgb, ll, 1.5, nu, 12 if L <= 16 else 5, prec)


def test_relaxation_gap_and_dice_on_the_tiny_workload(ctx):
    """The rounded solution within 1 % of the dual bound (the paper's
    typical figure), and the boundary term raises the agreement with the
    ground-truth regions over the pointwise most likely label."""
    w = make_config(0)
    masks, _, _ = oracle.full_masks(w)
    ll = oracle.label_loglik(w.rgb, masks, w.k, w.sample_pix, w.sample_label, w.L)
    lab, _, st = _run(ctx, w.rgb, ll, 1.0, 0.0, 600, "fp32")
    assert st["binary"] - st["dual"] <= 0.01 * abs(st["dual"])
    d0 = osg.dice(np.argmax(ll, 1).reshape(w.H, w.W), w.region, w.L).mean()
    d1 = osg.dice(lab, w.region, w.L).mean()
    assert d1 >= d0


def test_edge_weight_parity(ctx):
    w = make_config(1)
    g, gm = ctx.edge_weight(dev(w.rgb))
    g_ref, gm_ref = osg.edge_weight(w.rgb)
    assert abs(gm - gm_ref) <= 1e-12 * gm_ref
    np.testing.assert_allclose(g.cpu().numpy(), g_ref, rtol=2 ** -23, atol=0)
    g5, gm5 = ctx.edge_weight(dev(w.rgb), 5.0)
    assert gm5 == 5.0
    np.testing.assert_allclose(g5.cpu().numpy(), osg.edge_weight(w.rgb, 5.0)[0], rtol=2 ** -23, atol=0)


def test_errors(ctx):
    from paper_1312_4746_amd import CosparseError, SegmentParams
    w = make_config(0)
    ll = dev(np.zeros((w.N, w.L), np.float32))
    rgb = dev(w.rgb)
    for prm in (SegmentParams(lam=-1.0), SegmentParams(nu=-0.1), SegmentParams(iterations=-1),
                SegmentParams(lam=float("nan"))):
        with pytest.raises(CosparseError) as e:
            ctx.segment(rgb, ll, prm)
        assert e.value.code == 1
    # a constant image has no mean gradient: the metric needs an explicit gamma
    flat = dev(np.full((3, 8, 9), 0.3, np.float32))
    with pytest.raises(CosparseError) as e:
        ctx.segment(flat, dev(np.zeros((72, 2), np.float32)), SegmentParams())
    assert e.value.code == 1
    lab, _, st = ctx.segment(flat, dev(np.zeros((72, 2), np.float32)), SegmentParams(gamma=1.0, iterations=5))
    assert st["gamma"] == 1.0
