"""Parity of the joint data term (eq:joined: colour/location Parzen density
times the texture posterior against the label representatives) on the HIP
path, through the C-ABI, with the FP64 oracle: log-likelihoods within
1e-5 * max(1, |l|), on full images (the matrix-core route the benchmark
times), pixel subsets (the exact route) and the degenerate cases of the
majority vote."""
import dataclasses

import numpy as np
import pytest
import torch

import oracle
from workloads import make_config, make_workload

pytestmark = pytest.mark.gpu

LL_TOL = 1e-5


@pytest.fixture(scope="module")
def ctx():
    from paper_1312_4746_amd import Context
    c = Context(0)
    yield c
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _check(got, ref):
    got = got.astype(np.float64)
    tol = LL_TOL * np.maximum(1.0, np.abs(ref))
    err = np.abs(got - ref)
    assert np.all(np.isfinite(got))
    assert np.all(err <= tol), (float((err / tol).max()), np.unravel_index(np.argmax(err / tol), err.shape))


def _both(ctx, w, masks, pix=None, ref_pix=None, **kw):
    from paper_1312_4746_amd import LoglikParams
    prm = LoglikParams(alpha_rho=kw.get("alpha_rho", w.alpha_rho), sigma_c=kw.get("sigma_c", w.sigma_c),
                       beta_scale=kw.get("beta_scale", w.beta_scale),
                       rho_floor_px=kw.get("rho_floor", w.rho_floor_px),
                       normalise=kw.get("normalise", False),
                       colour_levels=kw.get("colour_levels", w.colour_levels))
    got = ctx.label_loglik(dev(w.rgb), dev(masks.view(np.int64)), w.k, dev(w.sample_pix),
                           dev(w.sample_label), w.L, prm,
                           pix_subset=None if pix is None else dev(np.asarray(pix, np.int32)),
                           joint=True).cpu().numpy()
    rp = pix if ref_pix is None else ref_pix
    ref = oracle.label_loglik(w.rgb, masks, w.k, w.sample_pix, w.sample_label, w.L,
                              alpha_rho=prm.alpha_rho, sigma_c=prm.sigma_c, beta_scale=prm.beta_scale,
                              rho_floor=prm.rho_floor_px, normalise=prm.normalise, pix=rp, joint=True)
    return got, ref


CASES = [
    dict(name="p3k1", H=9, W=11, R=2, p=3, k=1),
    dict(name="p5k50", H=64, W=64, R=3, p=5, k=50),
    dict(name="p7k98_ragged", H=37, W=70, R=4, p=7, k=98),
    dict(name="p9k64", H=33, W=129, R=3, p=9, k=64),
    dict(name="p11k242", H=40, W=66, R=5, p=11, k=242),
    dict(name="p15k256", H=31, W=65, R=3, p=15, k=256),
]


def test_joint_tiny_config_full(ctx):
    w = make_config(0)
    masks, _, _ = oracle.full_masks(w)
    got, ref = _both(ctx, w, masks)
    _check(got, ref)


@pytest.mark.parametrize("case", CASES, ids=lambda c: c["name"])
def test_joint_small_cases_full_and_subset(ctx, case):
    c = dict(case)
    name = c.pop("name")
    w = make_workload(name, seed=7, per_region=6, **c)
    masks, _, _ = oracle.full_masks(w)
    got, ref = _both(ctx, w, masks)
    _check(got, ref)
    pix = np.array([w.N - 1, 0, 3, 3, w.N // 2], np.int32)
    got, ref = _both(ctx, w, masks, pix=pix)
    _check(got, ref)


@pytest.mark.parametrize("kw", [dict(normalise=True), dict(beta_scale=1e30, rho_floor=40.0),
                                dict(alpha_rho=0.7, sigma_c=0.2, beta_scale=0.25)])
def test_joint_parameter_forms(ctx, kw):
    w = make_config(0)
    masks, _, _ = oracle.full_masks(w)
    got, ref = _both(ctx, w, masks, **kw)
    _check(got, ref)
    if kw.get("normalise"):
        np.testing.assert_allclose(np.exp(got.astype(np.float64)).sum(1), 1.0, atol=1e-5)


def test_joint_majority_ties_and_tiny_labels(ctx):
    """Random co-supports, labels of 1, 2, 3 and 4 samples: even labels tie
    on many bits (ties count in), a one-sample label's representative is that
    sample's co-support."""
    rng = np.random.default_rng(17)
    H, W, k = 12, 13, 77
    N = H * W
    bits = rng.random((N, k)) < 0.5
    masks = np.zeros((N, 2), np.uint64)
    for j in range(k):
        masks[:, j // 64] |= bits[:, j].astype(np.uint64) << np.uint64(j % 64)
    w = make_workload("ties", H=H, W=W, R=2, p=3, k=k, seed=3, per_region=4)
    sp = rng.choice(N, 10, replace=False).astype(np.int32)
    sl = np.array([0, 1, 1, 2, 2, 2, 3, 3, 3, 3], np.int32)
    w = dataclasses.replace(w, sample_pix=sp, sample_label=sl, L=4)
    got, ref = _both(ctx, w, masks)
    _check(got, ref)


def test_joint_bsds_full_image_sampled(ctx):
    """481 x 321, k = 98, 10 labels, 7,720 samples: the launch configuration
    the benchmark times, checked on sampled pixels (corners included)."""
    w = make_config(1)
    masks, _, _ = oracle.full_masks(w)
    rng = np.random.default_rng(31)
    pix = np.unique(np.concatenate([rng.choice(w.N, 1200, replace=False),
                                    [0, w.W - 1, w.N - w.W, w.N - 1]])).astype(np.int32)
    got, ref = _both(ctx, w, masks, ref_pix=pix)
    _check(got[pix], ref)


def test_joint_large_full_image_sampled(ctx):
    """1024 x 1024, k = 242, 16 labels, 50,000 samples; masks from the library
    (bit-exact with the oracle on every smaller case)."""
    w = make_config(3)
    rgb = dev(w.rgb)
    a = ctx.analyze_patches(rgb, w.p, w.mask_sigma, dev(w.omega))
    tau = ctx.tau_median(rgb, w.p, w.mask_sigma, dev(w.omega), a, 0.1)
    masks = ctx.cosupport(rgb, w.p, w.mask_sigma, dev(w.omega), tau, alpha=a).cpu().numpy().view(np.uint64)
    rng = np.random.default_rng(32)
    pix = np.unique(np.concatenate([rng.choice(w.N, 300, replace=False), [0, w.N - 1]])).astype(np.int32)
    got, ref = _both(ctx, w, masks, ref_pix=pix)
    _check(got[pix], ref)


def test_joint_errors_and_empty_subset(ctx):
    from paper_1312_4746_amd import LoglikParams
    w = make_config(0)
    masks, _, _ = oracle.full_masks(w)
    from paper_1312_4746_amd.binding import CosparseError
    with pytest.raises(CosparseError) as e:
        ctx.label_loglik(dev(w.rgb), dev(masks.view(np.int64)), w.k, dev(w.sample_pix),
                         dev(w.sample_label), w.L + 1, LoglikParams(), joint=True)
    assert e.value.code == 2
    out = ctx.label_loglik(dev(w.rgb), dev(masks.view(np.int64)), w.k, dev(w.sample_pix),
                           dev(w.sample_label), w.L, LoglikParams(),
                           pix_subset=dev(np.zeros(0, np.int32)), joint=True)
    assert out.shape == (0, w.L)
