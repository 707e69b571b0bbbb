"""Parity of the joint data term with smooth co-supports (eq:map_tsm, eq:tsm,
eq:approx_cosupp) on the HIP path, through the C-ABI, with the FP64 oracle:
both sides take the same FP32 analysed vectors; log-likelihoods within
1e-5 * max(1, |l|)."""
import dataclasses

import numpy as np
import pytest
import torch

import oracle
from workloads import make_config, make_workload

pytestmark = pytest.mark.gpu

LL_TOL = 1e-5
SIGMA = 0.01


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


def _both(ctx, w, a32, pix=None, ref_pix=None, sigma=SIGMA, **kw):
    from paper_1312_4746_amd import LoglikParams
    prm = LoglikParams(alpha_rho=kw.get("alpha_rho", w.alpha_rho), sigma_c=kw.get("sigma_c", w.sigma_c),
                       beta_scale=kw.get("beta_scale", w.beta_scale),
                       rho_floor_px=kw.get("rho_floor", w.rho_floor_px),
                       normalise=kw.get("normalise", False),
                       colour_levels=kw.get("colour_levels", w.colour_levels))
    got = ctx.label_loglik_soft(dev(w.rgb), dev(a32), sigma, dev(w.sample_pix), dev(w.sample_label), w.L,
                                prm, pix_subset=None if pix is None else dev(np.asarray(pix, np.int32)))
    rp = pix if ref_pix is None else ref_pix
    ref = oracle.label_loglik_soft(w.rgb, a32.astype(np.float64), sigma, w.sample_pix, w.sample_label, w.L,
                                   alpha_rho=prm.alpha_rho, sigma_c=prm.sigma_c, beta_scale=prm.beta_scale,
                                   rho_floor=prm.rho_floor_px, normalise=prm.normalise, pix=rp)
    return got.cpu().numpy(), ref


def _alpha32(w):
    return oracle.analyze(w.rgb, w.p, w.mask_sigma, w.omega).astype(np.float32)


def _library_alpha(ctx, w):
    return ctx.analyze_patches(dev(w.rgb), w.p, w.mask_sigma, dev(w.omega)).cpu().numpy()


CASES = [
    dict(name="p3k1", H=9, W=11, R=2, p=3, k=1),
    dict(name="p5k50", H=64, W=64, R=3, p=5, k=50),
    dict(name="p7k98_ragged", H=37, W=70, R=4, p=7, k=98),
    dict(name="p11k242", H=40, W=66, R=5, p=11, k=242),
    dict(name="p15k256", H=31, W=65, R=3, p=15, k=256),
    dict(name="p5k30_L20", H=40, W=50, R=20, p=5, k=30),
]


def test_soft_tiny_config_full(ctx):
    w = make_config(0)
    got, ref = _both(ctx, w, _alpha32(w))
    _check(got, ref)


@pytest.mark.parametrize("case", CASES, ids=lambda c: c["name"])
def test_soft_small_cases_full_and_subset(ctx, case):
    c = dict(case)
    name = c.pop("name")
    w = make_workload(name, seed=9, per_region=5, **c)
    a32 = _alpha32(w)
    got, ref = _both(ctx, w, a32)
    _check(got, ref)
    pix = np.array([w.N - 1, 0, 7, 7, w.N // 3], np.int32)
    got, ref = _both(ctx, w, a32, pix=pix)
    _check(got, ref)


@pytest.mark.parametrize("kw", [dict(normalise=True), dict(sigma=0.05, beta_scale=0.3),
                                dict(alpha_rho=0.7, sigma_c=0.2, rho_floor=3.0)])
def test_soft_parameter_forms(ctx, kw):
    w = make_config(0)
    kw = dict(kw)
    sigma = kw.pop("sigma", SIGMA)
    got, ref = _both(ctx, w, _alpha32(w), sigma=sigma, **kw)
    _check(got, ref)
    if kw.get("normalise"):
        np.testing.assert_allclose(np.exp(got.astype(np.float64)).sum(1), 1.0, atol=1e-5)


def test_soft_even_and_tiny_labels(ctx):
    """Labels of 1, 2, 3 and 4 samples (upper median of even counts)."""
    rng = np.random.default_rng(23)
    w = make_workload("tiny", H=12, W=13, R=2, p=3, k=45, seed=4, per_region=4)
    a32 = (rng.standard_normal((w.N, w.k)) * 0.1).astype(np.float32)
    sp = rng.choice(w.N, 10, replace=False).astype(np.int32)
    sl = np.array([0, 1, 1, 2, 2, 2, 3, 3, 3, 3], np.int32)
    w = dataclasses.replace(w, sample_pix=sp, sample_label=sl, L=4)
    got, ref = _both(ctx, w, a32)
    _check(got, ref)


def test_soft_bsds_full_image_sampled(ctx):
    """481 x 321, k = 98, 10 labels, 7,720 samples, sigma = 0.01 as in the
    paper's experiments; the library's own analysed vectors."""
    w = make_config(1)
    a32 = _library_alpha(ctx, w)
    rng = np.random.default_rng(41)
    pix = np.unique(np.concatenate([rng.choice(w.N, 1200, replace=False),
                                    [0, w.W - 1, w.N - w.W, w.N - 1]])).astype(np.int32)
    got, ref = _both(ctx, w, a32, ref_pix=pix)
    _check(got[pix], ref)


def test_soft_large_full_image_sampled(ctx):
    """1024 x 1024, k = 242, 16 labels, 50,000 samples."""
    w = make_config(3)
    a32 = _library_alpha(ctx, w)
    rng = np.random.default_rng(42)
    pix = np.unique(np.concatenate([rng.choice(w.N, 300, replace=False), [0, w.N - 1]])).astype(np.int32)
    got, ref = _both(ctx, w, a32, ref_pix=pix)
    _check(got[pix], ref)


def test_soft_errors(ctx):
    from paper_1312_4746_amd import LoglikParams
    from paper_1312_4746_amd.binding import CosparseError
    w = make_config(0)
    a = dev(_alpha32(w))
    for sigma in (0.0, -1.0, float("inf")):
        with pytest.raises(CosparseError) as e:
            ctx.label_loglik_soft(dev(w.rgb), a, sigma, dev(w.sample_pix), dev(w.sample_label), w.L,
                                  LoglikParams())
        assert e.value.code == 1
    with pytest.raises(CosparseError) as e:
        ctx.label_loglik_soft(dev(w.rgb), a, SIGMA, dev(w.sample_pix), dev(w.sample_label), w.L + 1,
                              LoglikParams())
    assert e.value.code == 2
    out = ctx.label_loglik_soft(dev(w.rgb), a, SIGMA, dev(w.sample_pix), dev(w.sample_label), w.L,
                                LoglikParams(), pix_subset=dev(np.zeros(0, np.int32)))
    assert out.shape == (0, w.L)
