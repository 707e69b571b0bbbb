"""Parity of the HIP path (through the C-ABI) with the FP64 oracle.

Bars: co-support masks, TSM counts and tau bit-exact; analysed vectors
within the proven per-row error bound of their precision; log-likelihoods
within 1e-5 * max(1, |l|) of the oracle.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from workloads import make_config, make_workload, quantise_colours

pytestmark = pytest.mark.gpu

LL_TOL = 1e-5


@pytest.fixture(scope="module")
def ctx():
    from paper_1312_4746_amd import Context
    c = Context(0)
    yield c
    c.close()


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def masks_u64(t):
    return t.cpu().numpy().view(np.uint64)


def bound_coef(prec, n):
    u = 2.0 ** -24
    if prec == "bf16":
        return 2.0 ** -7 + 2.0 ** -15 + 2 * (n + 4) * u
    return 2 * (n + 4) * u


def gpu_masks(ctx, w, tau, prec="fp32", margin=-1.0, stats=False, alpha=None):
    return ctx.cosupport(dev(w.rgb), w.p, w.mask_sigma, dev(w.omega), tau, margin=margin,
                         precision=prec, stats=stats, alpha=alpha)


SMALL_CASES = [
    dict(name="p3k1", H=9, W=11, R=2, p=3, k=1),
    dict(name="p5k50", H=64, W=64, R=3, p=5, k=50),
    dict(name="p7k98_ragged", H=37, W=70, R=4, p=7, k=98),
    dict(name="p9k64", H=33, W=129, R=3, p=9, k=64),
    dict(name="p11k242", H=40, W=66, R=5, p=11, k=242),
    dict(name="p15k256", H=31, W=65, R=3, p=15, k=256),
]


def _small(case, seed=7):
    c = dict(case)
    name = c.pop("name")
    return make_workload(name, seed=seed, per_region=6, **c)


@pytest.mark.parametrize("case", SMALL_CASES, ids=lambda c: c["name"])
@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_analyze_within_proven_bound(ctx, case, prec):
    w = _small(case)
    a_gpu = ctx.analyze_patches(dev(w.rgb), w.p, w.mask_sigma, dev(w.omega), precision=prec)
    a_ref = oracle.analyze(w.rgb, w.p, w.mask_sigma, w.omega)
    err = np.abs(a_gpu.cpu().numpy().astype(np.float64) - a_ref)
    rown = np.linalg.norm(w.omega.astype(np.float64), axis=1)
    bound = bound_coef(prec, w.n) * rown[None, :] + 2.0 ** -100
    assert np.all(err <= bound), float((err / bound).max())
    # the bound is not vacuous: the rounding error is visible but far inside it
    assert err.max() > 0


@pytest.mark.parametrize("case", SMALL_CASES, ids=lambda c: c["name"])
@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_tau_and_masks_bit_exact(ctx, case, prec):
    w = _small(case)
    a_ref = oracle.analyze(w.rgb, w.p, w.mask_sigma, w.omega)
    tau_ref, _ = oracle.tau_median(a_ref, 0.1)
    a_gpu = ctx.analyze_patches(dev(w.rgb), w.p, w.mask_sigma, dev(w.omega), precision=prec)
    tau = ctx.tau_median(dev(w.rgb), w.p, w.mask_sigma, dev(w.omega), a_gpu, 0.1, precision=prec)
    assert tau == tau_ref
    m_gpu, st = gpu_masks(ctx, w, tau, prec, stats=True)
    m_ref = oracle.cosupport(a_ref, tau_ref)
    assert np.array_equal(masks_u64(m_gpu), m_ref)
    # the same masks decided from the stored analysed vectors
    m_alpha, st_a = gpu_masks(ctx, w, tau, prec, stats=True, alpha=a_gpu)
    assert np.array_equal(masks_u64(m_alpha), m_ref)
    assert st_a["recomputed"] == st["recomputed"]


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_bsds_shape_tau_and_masks_bit_exact(ctx, prec):
    w = make_config(1)
    a_ref = oracle.analyze(w.rgb, w.p, w.mask_sigma, w.omega)
    tau_ref, _ = oracle.tau_median(a_ref, 0.1)
    a_gpu = ctx.analyze_patches(dev(w.rgb), w.p, w.mask_sigma, dev(w.omega), precision=prec)
    tau = ctx.tau_median(dev(w.rgb), w.p, w.mask_sigma, dev(w.omega), a_gpu, 0.1, precision=prec)
    assert tau == tau_ref
    m_gpu, st = gpu_masks(ctx, w, tau, prec, stats=True)
    m_ref = oracle.cosupport(a_ref, tau_ref)
    assert np.array_equal(masks_u64(m_gpu), m_ref)
    assert st["recomputed"] > 0
    m_alpha, st_a = gpu_masks(ctx, w, tau, prec, stats=True, alpha=a_gpu)
    assert np.array_equal(masks_u64(m_alpha), m_ref)
    assert st_a["recomputed"] == st["recomputed"]


@pytest.mark.parametrize("case", [SMALL_CASES[1], SMALL_CASES[2], SMALL_CASES[4]], ids=lambda c: c["name"])
@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_cosupport_median_matches_separate_calls(ctx, case, prec):
    """The enqueue-only co-support call gives the oracle's tau and masks and
    the same analysed vectors as the separate calls; two calls in a row with
    different images leave no state behind."""
    for seed in (7, 8):
        w = _small(case, seed=seed)
        a_ref = oracle.analyze(w.rgb, w.p, w.mask_sigma, w.omega)
        tau_ref, _ = oracle.tau_median(a_ref, 0.1)
        alpha, m, tau_d = ctx.cosupport_median(dev(w.rgb), w.p, w.mask_sigma, dev(w.omega), 0.1, precision=prec)
        assert float(tau_d.item()) == tau_ref
        assert np.array_equal(masks_u64(m), oracle.cosupport(a_ref, tau_ref))
        a_sep = ctx.analyze_patches(dev(w.rgb), w.p, w.mask_sigma, dev(w.omega), precision=prec)
        assert torch.equal(alpha, a_sep.view(alpha.shape))


def test_cosupport_median_bsds_shape_and_zero_image(ctx):
    w = make_config(1)
    a_ref = oracle.analyze(w.rgb, w.p, w.mask_sigma, w.omega)
    tau_ref, _ = oracle.tau_median(a_ref, 0.1)
    _, m, tau_d = ctx.cosupport_median(dev(w.rgb), w.p, w.mask_sigma, dev(w.omega), 0.1)
    assert float(tau_d.item()) == tau_ref
    assert np.array_equal(masks_u64(m), oracle.cosupport(a_ref, tau_ref))
    # every entry is a candidate of the exact selection (all |a| = 0)
    rgb = np.zeros((3, 20, 21), np.float32)
    om = np.random.default_rng(0).standard_normal((70, 25)).astype(np.float32)
    _, m0, t0 = ctx.cosupport_median(dev(rgb), 5, 1.25, dev(om), 0.1)
    assert float(t0.item()) == 0.0
    mm = masks_u64(m0)
    assert np.all(mm[:, 0] == np.uint64(0xFFFFFFFFFFFFFFFF))
    assert np.all(mm[:, 1] == np.uint64(63))


@pytest.mark.parametrize("period", [2, 3])
@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_tau_and_masks_with_heavy_ties(ctx, period, prec):
    """A degenerate image for the exact selection: vertical stripes of period
    2 or 3 on 256 x 256 pixels, k = 242, so that the patches repeat and the
    few analysed values near the median each occur tens of thousands of times
    (about 63 000 candidates in three values, or 21 000 in two).  The list
    exceeds the ranked selection's limit, and the radix passes meet more keys
    sharing a digit than the selection keeps in LDS; tau and the masks of the
    separate and the fused calls against the oracle, bit for bit."""
    import dataclasses
    w = make_workload("ties", H=256, W=256, R=2, p=11, k=242, seed=41, per_region=10)
    x = np.arange(w.W)
    pat = (x % period == 0).astype(np.float32)
    rgb = pat[None, None, :] * np.array([0.8, 0.5, 0.2], np.float32)[:, None, None] + np.float32(0.1)
    w = dataclasses.replace(w, rgb=np.ascontiguousarray(np.broadcast_to(rgb, (3, w.H, w.W))))
    a_ref = oracle.analyze(w.rgb, w.p, w.mask_sigma, w.omega)
    tau_ref, _ = oracle.tau_median(a_ref, 0.1)
    m_ref = oracle.cosupport(a_ref, tau_ref)
    a_gpu = ctx.analyze_patches(dev(w.rgb), w.p, w.mask_sigma, dev(w.omega), precision=prec)
    tau = ctx.tau_median(dev(w.rgb), w.p, w.mask_sigma, dev(w.omega), a_gpu, 0.1, precision=prec)
    assert tau == tau_ref
    assert np.array_equal(masks_u64(gpu_masks(ctx, w, tau, prec)), m_ref)
    _, m, tau_d = ctx.cosupport_median(dev(w.rgb), w.p, w.mask_sigma, dev(w.omega), 0.1, precision=prec)
    assert float(tau_d.item()) == tau_ref
    assert np.array_equal(masks_u64(m), m_ref)


def test_bf16_stated_margin_reports_mismatches(ctx):
    """Precision form at the stated margin 2^-8 tau: entries outside it are
    decided by the BF16 value; the mismatch count is reported, and the proven
    margin drives it to zero (checked above)."""
    w = make_config(2)
    a_ref = oracle.analyze(w.rgb, w.p, w.mask_sigma, w.omega)
    tau, _ = oracle.tau_median(a_ref, 0.1)
    m_ref = oracle.cosupport(a_ref, tau)
    m_gpu, st = gpu_masks(ctx, w, tau, "bf16", margin=2.0 ** -8 * tau, stats=True)
    _, st_p = gpu_masks(ctx, w, tau, "bf16", stats=True)
    diff = np.bitwise_xor(masks_u64(m_gpu), m_ref)
    mism = int(np.unpackbits(diff.view(np.uint8)).sum())
    assert st["recomputed"] > 0
    # a mismatched bit is an entry outside the stated margin (so not recomputed)
    # whose BF16 value lies on the other side of tau from its exact value: it
    # lies within the proven BF16 error bound of tau (so the proven margin
    # recomputes it).  Hence the count is at most the entries that only the
    # proven margin recomputes, and each one is within that bound of tau.
    assert 0 < mism <= st_p["recomputed"] - st["recomputed"], (mism, st, st_p)
    rown = np.linalg.norm(w.omega.astype(np.float64), axis=1)
    rows, words = np.nonzero(diff)
    for r, q in zip(rows, words):
        v = int(diff[r, q])
        while v:
            j = q * 64 + (v & -v).bit_length() - 1
            v &= v - 1
            assert abs(abs(a_ref[r, j]) - tau) <= bound_coef("bf16", w.n) * rown[j], (r, j)
    # same decisions from the stored BF16 analysed vectors
    a_gpu = ctx.analyze_patches(dev(w.rgb), w.p, w.mask_sigma, dev(w.omega), precision="bf16")
    m_alpha = gpu_masks(ctx, w, tau, "bf16", margin=2.0 ** -8 * tau, alpha=a_gpu)
    assert np.array_equal(masks_u64(m_alpha), masks_u64(m_gpu))


def test_zero_image_full_cosupport(ctx):
    rgb = np.zeros((3, 20, 21), np.float32)
    om = np.random.default_rng(0).standard_normal((70, 25)).astype(np.float32)
    m = ctx.cosupport(dev(rgb), 5, 1.25, dev(om), 0.0)
    mm = masks_u64(m)
    assert np.all(mm[:, 0] == np.uint64(0xFFFFFFFFFFFFFFFF))
    assert np.all(mm[:, 1] == np.uint64(63))


@pytest.mark.parametrize("k", [1, 50, 63, 64, 65, 98, 242, 256])
def test_texture_similarity_bit_exact(ctx, k):
    rng = np.random.default_rng(k)
    nw = (k + 63) // 64
    for na, nb in [(1, 1), (70, 129), (130, 3)]:
        A = rng.integers(0, 2 ** 63, size=(na, nw), dtype=np.int64).view(np.uint64)
        B = rng.integers(0, 2 ** 63, size=(nb, nw), dtype=np.int64).view(np.uint64)
        A[0] = 0
        out = ctx.texture_similarity(dev(A.view(np.int64)), dev(B.view(np.int64)), k)
        # padding bits beyond k are ignored by definition: clear them for the oracle
        if k % 64:
            A[:, -1] &= np.uint64((1 << (k % 64)) - 1)
            B[:, -1] &= np.uint64((1 << (k % 64)) - 1)
        assert np.array_equal(out.cpu().numpy(), oracle.tsm(A, B, k))


def test_texture_similarity_symmetric_and_zero_diagonal(ctx):
    w = make_config(0)
    m, _, _ = oracle.full_masks(w)
    md = dev(m.view(np.int64))
    T = ctx.texture_similarity(md[:300], md[:300], w.k).cpu().numpy()
    assert np.array_equal(T, T.T) and np.all(np.diag(T) == 0)


def _ll_check(got, ref):
    got = got.astype(np.float64)
    tol = LL_TOL * np.maximum(1.0, np.abs(ref))
    err = np.abs(got - ref)
    assert np.all(np.isfinite(got))
    assert np.all(err <= tol), (float((err / tol).max()), np.unravel_index(np.argmax(err / tol), err.shape))


def _loglik_both(ctx, w, masks, pix=None, **kw):
    from paper_1312_4746_amd import LoglikParams
    prm = LoglikParams(alpha_rho=kw.get("alpha_rho", w.alpha_rho), sigma_c=kw.get("sigma_c", w.sigma_c),
                       beta_scale=kw.get("beta_scale", w.beta_scale),
                       rho_floor_px=kw.get("rho_floor", w.rho_floor_px),
                       normalise=kw.get("normalise", False),
                       colour_levels=kw.get("colour_levels", w.colour_levels))
    got = ctx.label_loglik(dev(w.rgb), dev(masks.view(np.int64)), w.k, dev(w.sample_pix),
                           dev(w.sample_label), w.L, prm,
                           pix_subset=None if pix is None else dev(np.asarray(pix, np.int32)))
    ref = oracle.label_loglik(w.rgb, masks, w.k, w.sample_pix, w.sample_label, w.L,
                              alpha_rho=prm.alpha_rho, sigma_c=prm.sigma_c, beta_scale=prm.beta_scale,
                              rho_floor=prm.rho_floor_px, normalise=prm.normalise, pix=pix)
    return got.cpu().numpy(), ref


def test_loglik_tiny_config_full(ctx):
    w = make_config(0)
    masks, _, _ = oracle.full_masks(w)
    got, ref = _loglik_both(ctx, w, masks)
    _ll_check(got, ref)


@pytest.mark.parametrize("case", SMALL_CASES, ids=lambda c: c["name"])
@pytest.mark.parametrize("levels", [0, 255, 17])
def test_loglik_small_cases_full(ctx, case, levels):
    """Float colours (levels 0) and colours at 255 or 17 levels per channel,
    whose squared distances the matrix-core kernel forms as exact integers."""
    w = _small(case)
    if levels:
        w.rgb = quantise_colours(w.rgb, levels)
    masks, _, _ = oracle.full_masks(w)
    got, ref = _loglik_both(ctx, w, masks, colour_levels=levels)
    _ll_check(got, ref)


def test_loglik_colour_levels_match_float_colours(ctx):
    """On an 8-bit image the colour-level route and the float-colour route
    give the same rows within FP32 rounding of the exponents (both inside the
    oracle bound), on the tile grid and on a pixel list."""
    w = make_config(1)
    masks, _, _ = oracle.full_masks(w)
    rng = np.random.default_rng(5)
    pix = rng.choice(w.N, 2048, replace=False).astype(np.int32)
    for sub in (None, pix):
        a, ref = _loglik_both(ctx, w, masks, pix=sub, colour_levels=255)
        b, _ = _loglik_both(ctx, w, masks, pix=sub, colour_levels=0)
        if sub is not None:
            _ll_check(a, ref)
            _ll_check(b, ref)
        np.testing.assert_allclose(a, b, rtol=2e-5, atol=2e-5)


def test_loglik_colour_levels_errors(ctx):
    """colour_levels outside 0..255 is an argument error; with the input check
    on, a colour that is no multiple of 1/n, or lies above 255/n, is too."""
    from paper_1312_4746_amd import CosparseError, LoglikParams
    w = make_config(0)
    masks, _, _ = oracle.full_masks(w)
    args = (dev(masks.view(np.int64)), w.k, dev(w.sample_pix), dev(w.sample_label), w.L)
    for n in (-1, 256):
        with pytest.raises(CosparseError) as e:
            ctx.label_loglik(dev(w.rgb), *args, LoglikParams(colour_levels=n))
        assert e.value.code == 1
    ctx.set_check_finite(True)
    try:
        ctx.label_loglik(dev(w.rgb), *args, LoglikParams(colour_levels=255))  # 8-bit image: accepted
        for bad in (0.5 / 255, 1.0 + 1.0 / 255):
            rgb = w.rgb.copy()
            rgb[1, 3, 4] = bad
            with pytest.raises(CosparseError) as e:
                ctx.label_loglik(dev(rgb), *args, LoglikParams(colour_levels=255))
            assert e.value.code == 1
        rgb = w.rgb.copy()
        rgb[0, 0, 0] = np.nan
        with pytest.raises(CosparseError) as e:
            ctx.label_loglik(dev(rgb), *args, LoglikParams(colour_levels=255))
        assert e.value.code == 5
    finally:
        ctx.set_check_finite(False)


def test_loglik_bsds_shape_subset(ctx):
    w = make_config(1)
    masks, _, _ = oracle.full_masks(w)
    rng = np.random.default_rng(3)
    pix = np.concatenate([rng.choice(w.N, 1500, replace=False), [0, w.N - 1, 5, 5]]).astype(np.int32)
    got, ref = _loglik_both(ctx, w, masks, pix=pix)
    _ll_check(got, ref)


@pytest.mark.parametrize("kw", [dict(normalise=True), dict(beta_scale=1e30, rho_floor=40.0),
                                dict(alpha_rho=0.7, sigma_c=0.2, beta_scale=3.0)])
def test_loglik_parameter_forms(ctx, kw):
    w = make_config(0)
    masks, _, _ = oracle.full_masks(w)
    got, ref = _loglik_both(ctx, w, masks, **kw)
    _ll_check(got, ref)
    if kw.get("normalise"):
        np.testing.assert_allclose(np.exp(got.astype(np.float64)).sum(1), 1.0, atol=1e-5)


def test_loglik_overflow_fixup_case(ctx):
    """A pixel whose nearest sample matches badly while a farther sample
    matches exactly: the first reference overflows and the exact-max pass
    must take over."""
    H, W = 16, 16
    rgb = np.full((3, H, W), 0.5, np.float32)
    x = 8 * W + 8
    near, far = 8 * W + 9, 8 * W + 11
    rgb[:, 8, 9] = 1.5          # colour distance 1 per channel: about 600 nats worse
    masks = np.zeros((H * W, 1), np.uint64)
    w = make_workload("fix", H=H, W=W, R=1, p=3, k=8, seed=1, per_region=2)
    w.rgb = rgb
    w.sample_pix = np.array([near, far, 0], np.int32)
    w.sample_label = np.array([0, 0, 0], np.int32)
    w.L = 1
    w.k = 8
    got, ref = _loglik_both(ctx, w, masks, pix=np.array([x, x + 1, 0], np.int32))
    _ll_check(got, ref)


@pytest.mark.parametrize("levels", [0, 255])
def test_loglik_overflow_case_full_image(ctx, levels):
    """Same construction on the full-image path (texture term on the matrix
    cores): the reference must move up by the dynamic rescale.  With colour
    levels the colours are 0 and 1 (the same distance 1 per channel)."""
    H, W = 16, 24
    rgb = np.full((3, H, W), 0.5 if levels == 0 else 0.0, np.float32)
    rgb[:, 8, 9] = 1.5 if levels == 0 else 1.0
    rgb[:, 3, 20] = -0.7 if levels == 0 else 1.0
    w = make_workload("fix2", H=H, W=W, R=1, p=3, k=8, seed=1, per_region=2)
    w.rgb = rgb
    w.sample_pix = np.array([8 * W + 9, 8 * W + 11, 0, 3 * W + 20, 3 * W + 23], np.int32)
    w.sample_label = np.array([0, 0, 0, 1, 1], np.int32)
    w.L = 2
    w.k = 8
    masks = np.zeros((H * W, 1), np.uint64)
    masks[::3, 0] = np.uint64(0b10110)
    got, ref = _loglik_both(ctx, w, masks, colour_levels=levels)
    _ll_check(got, ref)


def test_loglik_empty_subset_and_single_sample_labels(ctx):
    w = make_workload("one", H=20, W=23, R=3, p=5, k=40, seed=3, per_region=1)
    masks, _, _ = oracle.full_masks(w)
    got, ref = _loglik_both(ctx, w, masks)
    _ll_check(got, ref)
    got, ref = _loglik_both(ctx, w, masks, pix=np.zeros(0, np.int32))
    assert got.shape == (0, w.L)


def test_loglik_errors(ctx):
    from paper_1312_4746_amd import CosparseError, LoglikParams
    w = make_config(0)
    masks, _, _ = oracle.full_masks(w)
    args = (dev(w.rgb), dev(masks.view(np.int64)), w.k, dev(w.sample_pix))
    with pytest.raises(CosparseError) as e:
        ctx.label_loglik(*args, dev(w.sample_label), w.L + 1, LoglikParams())
    assert e.value.code == 2
    bad = w.sample_label.copy()
    bad[5] = 99
    with pytest.raises(CosparseError) as e:
        ctx.label_loglik(*args, dev(bad), w.L, LoglikParams())
    assert e.value.code == 1
    with pytest.raises(CosparseError) as e:
        ctx.label_loglik(*args, dev(w.sample_label), w.L, LoglikParams(),
                         pix_subset=dev(np.array([0, w.N], np.int32)))
    assert e.value.code == 1
    with pytest.raises(CosparseError) as e:
        ctx.label_loglik(*args, dev(w.sample_label), w.L, LoglikParams(sigma_c=0.0))
    assert e.value.code == 1


def test_patch_errors(ctx):
    from paper_1312_4746_amd import CosparseError
    w = make_config(0)
    for p, k in [(4, 50), (17, 50), (5, 257)]:
        om = np.zeros((k, p * p), np.float32)
        with pytest.raises(CosparseError) as e:
            ctx.analyze_patches(dev(w.rgb), p, 1.0, dev(om))
        assert e.value.code == 1
    with pytest.raises(CosparseError) as e:
        ctx.analyze_patches(dev(w.rgb), 5, 0.0, dev(w.omega))
    assert e.value.code == 1


def _full_image_sampled(ctx, w, masks, n_sample, seed):
    """The full-image (fast) path in the launch configuration the benchmark
    times, checked against the oracle on sampled pixels (border and corner
    pixels included)."""
    from paper_1312_4746_amd import LoglikParams
    prm = LoglikParams(alpha_rho=w.alpha_rho, sigma_c=w.sigma_c, beta_scale=w.beta_scale,
                       rho_floor_px=w.rho_floor_px, colour_levels=w.colour_levels)
    got = ctx.label_loglik(dev(w.rgb), dev(masks.view(np.int64)), w.k, dev(w.sample_pix),
                           dev(w.sample_label), w.L, prm).cpu().numpy()
    rng = np.random.default_rng(seed)
    pix = np.unique(np.concatenate([rng.choice(w.N, n_sample, replace=False),
                                    [0, w.W - 1, w.N - w.W, w.N - 1], w.sample_pix[:8]])).astype(np.int32)
    ref = oracle.label_loglik(w.rgb, masks, w.k, w.sample_pix, w.sample_label, w.L, alpha_rho=prm.alpha_rho,
                              sigma_c=prm.sigma_c, beta_scale=prm.beta_scale, rho_floor=prm.rho_floor_px,
                              pix=pix)
    _ll_check(got[pix], ref)
    assert np.all(np.isfinite(got))
    return ctx.last_loglik_stats()


def test_loglik_bsds_full_image_fast_path(ctx):
    w = make_config(1)
    masks, _, _ = oracle.full_masks(w)
    st = _full_image_sampled(ctx, w, masks, 1500, 11)
    assert st["overflow_tiles"] == 0


def test_loglik_large_full_image_fast_path(ctx):
    """1024x1024, k = 242 (two 128-feature FP6 steps), 16 labels, 50,000 samples;
    the masks come from the library (bit-exact with the oracle at every
    smaller case above, p = 11 and k = 242 included)."""
    w = make_config(3)
    rgb = dev(w.rgb)
    a = ctx.analyze_patches(rgb, w.p, w.mask_sigma, dev(w.omega))
    tau = ctx.tau_median(rgb, w.p, w.mask_sigma, dev(w.omega), a, 0.1)
    m = ctx.cosupport(rgb, w.p, w.mask_sigma, dev(w.omega), tau, alpha=a)
    masks = masks_u64(m)
    _full_image_sampled(ctx, w, masks, 400, 12)


@pytest.mark.parametrize("levels", [0, 255])
def test_loglik_label_blocks_with_partial_last_block(ctx, levels):
    """The work order's label blocks when they do not divide the labels: five
    labels of 6 400 samples at k = 242 (100 stream chunks of 64 samples, 19 456
    B each, per label) give blocks of two labels within the 4 MiB budget, so
    the blocks are 2, 2 and 1 labels; 384 x 384 pixels make 1 152 pixel groups,
    144 per queue, of which 80 go block by block before the 64 taken label by
    label."""
    w = make_workload("blocks", H=384, W=384, R=5, p=11, k=242, seed=31, per_region=6400,
                      colour_levels=levels)
    counts = np.bincount(w.sample_label, minlength=w.L)
    chunk = 64 * 256 + 12 * 4 * 64
    assert np.all(counts == 6400) and 2 * 100 * chunk <= 4 << 20 < 3 * 100 * chunk
    masks, _, _ = oracle.full_masks(w)
    st = _full_image_sampled(ctx, w, masks, 500, 31)
    assert st["exact_tiles"] == 0


@pytest.mark.parametrize("shape", [(16, 2048), (2048, 12)], ids=["W2048", "H2048"])
def test_loglik_largest_coordinates_fast_path(ctx, shape):
    """Positions up to 2047 on the matrix-core path, whose location product is
    exact only below 2048: last row and column included in the samples."""
    import dataclasses
    H, W = shape
    w = make_workload("edge", H=H, W=W, R=2, p=5, k=40, seed=5, per_region=40)
    corners = np.array([W - 1, (H - 1) * W, H * W - 1], np.int32)
    sp = np.unique(np.concatenate([w.sample_pix, corners])).astype(np.int32)
    w = dataclasses.replace(w, sample_pix=sp, sample_label=w.region.ravel()[sp].astype(np.int32))
    masks, _, _ = oracle.full_masks(w)
    _full_image_sampled(ctx, w, masks, 600, 21)


def test_loglik_wide_image_exact_route(ctx):
    """Images wider than 2048 take the exact kernel on the full image."""
    w = make_workload("wide", H=10, W=2050, R=2, p=3, k=18, seed=6, per_region=30)
    masks, _, _ = oracle.full_masks(w)
    st = _full_image_sampled(ctx, w, masks, 600, 22)
    assert st == {"rescaled_chunks": 0, "overflow_tiles": 0, "exact_tiles": 0}


@pytest.mark.parametrize("k", [6, 7, 119, 120, 121, 124, 125, 244, 245])
@pytest.mark.parametrize("levels", [0, 255])
def test_loglik_feature_width_boundary(ctx, k, levels):
    """The texture features (k mask bits, then D + 1 slots each for |A| and |B|,
    D = ceil(floor(k/7) / 7) base-7 digits) fill one 128-wide FP6 step up to
    k = 120, two up to k = 244 and three above; k < 7 needs no digit.  Both
    colour routes."""
    w = make_workload(f"kb{k}", H=18, W=27, R=3, p=5, k=k, seed=k, per_region=8, colour_levels=levels)
    masks, _, _ = oracle.full_masks(w)
    got, ref = _loglik_both(ctx, w, masks)
    _ll_check(got, ref)


def test_two_contexts_interleaved(ctx):
    """Two contexts on one device, their calls interleaved: each context keeps
    its own device counters, label-count hand-over and work queues, so the
    results equal those of one context alone (bit for bit)."""
    from paper_1312_4746_amd import Context, LoglikParams
    ws = [make_workload("ctx_a", H=40, W=56, R=3, p=5, k=40, seed=21, per_region=20),
          make_workload("ctx_b", H=33, W=47, R=4, p=7, k=98, seed=22, per_region=15)]

    def run(c, w):
        rgb = dev(w.rgb)
        _, m, tau = c.cosupport_median(rgb, w.p, w.mask_sigma, dev(w.omega), 0.1)
        prm = LoglikParams(alpha_rho=w.alpha_rho, sigma_c=w.sigma_c, beta_scale=w.beta_scale,
                           rho_floor_px=w.rho_floor_px, colour_levels=w.colour_levels)
        ll = c.label_loglik(rgb, m, w.k, dev(w.sample_pix), dev(w.sample_label), w.L, prm)
        return float(tau.item()), m.cpu(), ll.cpu()

    ref = [run(ctx, w) for w in ws]
    other = Context(0)
    try:
        got = [run(other, ws[0]), run(ctx, ws[1]), run(other, ws[1]), run(ctx, ws[0]), run(other, ws[0])]
    finally:
        other.close()
    for (tau, m, ll), i in zip(got, (0, 1, 1, 0, 0)):
        assert tau == ref[i][0]
        assert torch.equal(m, ref[i][1])
        assert torch.equal(ll, ref[i][2])


@pytest.mark.parametrize("levels", [0, 255])
def test_loglik_overflow_retry_on_matrix_core_path(ctx, levels):
    """Sums that overflow inside a chunk are computed again on the matrix-core
    path with raised references (no hand-off to the exact kernel): every
    sample the reference is estimated from (the nearest one and four strided
    ones) is 0.8 off in every colour channel, about 550 log2 units below the
    two good samples at the corners (with colour levels: colours 0 and 0.8)."""
    H, W = 16, 24
    rgb = np.full((3, H, W), 0.5 if levels == 0 else 0.0, np.float32)
    bad = [(r, c) for r in range(6, 10) for c in range(7, 17)]  # 40 samples
    for r, c in bad:
        rgb[:, r, c] = 1.3 if levels == 0 else 204.0 / 255.0
    pix = [r * W + c for r, c in bad]
    pix[5] = 0              # good samples (colour 0.5) at indices 5 and 15 of the label,
    pix[15] = H * W - 1     # away from the strided probes 0, 10, 20, 30
    w = make_workload("retry", H=H, W=W, R=1, p=3, k=8, seed=1, per_region=2)
    w.rgb = rgb
    w.sample_pix = np.array(pix, np.int32)
    w.sample_label = np.zeros(len(pix), np.int32)
    w.L = 1
    w.k = 8
    w.colour_levels = levels
    masks = np.zeros((H * W, 1), np.uint64)
    got, ref = _loglik_both(ctx, w, masks)
    _ll_check(got, ref)
    st = ctx.last_loglik_stats()
    assert st["overflow_tiles"] > 0, st
    assert st["exact_tiles"] == 0, st


def _list_case():
    return make_workload("list", H=40, W=56, R=4, p=5, k=40, seed=31, per_region=20)


@pytest.mark.parametrize("n", [1023, 1024, 1061])
@pytest.mark.parametrize("levels", [0, 255])
def test_loglik_pixel_list_routes(ctx, n, levels):
    """Pixel subsets below 1024 entries take the exact kernel, from 1024 on the
    matrix-core kernel in tiles of 32 consecutive entries (1024: 32 whole
    tiles; 1061: a ragged last tile); duplicates and the corner pixels
    included.  On the matrix-core path every row equals the full-image
    result of its pixel bit for bit (float colours: the 16 x 16 kernel; 8-bit
    colours: the 32 x 32 one)."""
    w = _list_case()
    if levels:
        w.rgb = quantise_colours(w.rgb, levels)
        w.colour_levels = levels
    masks, _, _ = oracle.full_masks(w)
    rng = np.random.default_rng(n)
    pix = rng.integers(0, w.N, n).astype(np.int32)
    pix[:4] = [0, w.N - 1, 7, 7]
    got, ref = _loglik_both(ctx, w, masks, pix=pix)
    _ll_check(got, ref)
    st = ctx.last_loglik_stats()
    if n < 1024:
        assert st == {"rescaled_chunks": 0, "overflow_tiles": 0, "exact_tiles": 0}
        return
    assert st["exact_tiles"] == 0, st
    full, _ = _loglik_both(ctx, w, masks)
    assert np.array_equal(got, full[pix])


@pytest.mark.parametrize("levels", [0, 255])
def test_loglik_pixel_list_distance_rows(ctx, levels):
    """A list of at most an eighth of the pixels takes the distance
    transform's row pass per listed entry: its rows equal the full image's bit
    for bit (the distances, and the nearest samples that set each pixel's
    log-sum-exp reference, are those of the full pass, ties included), on the
    matrix-core path (3 000 entries with duplicates and the corners) and on
    the exact kernel (600 entries) against the oracle."""
    from paper_1312_4746_amd import LoglikParams
    w = make_workload("lrows", H=192, W=160, R=5, p=5, k=40, seed=33, per_region=25, colour_levels=levels)
    masks, _, _ = oracle.full_masks(w)
    prm = LoglikParams(alpha_rho=w.alpha_rho, sigma_c=w.sigma_c, beta_scale=w.beta_scale,
                       rho_floor_px=w.rho_floor_px, colour_levels=levels)
    args = (dev(w.rgb), dev(masks.view(np.int64)), w.k, dev(w.sample_pix), dev(w.sample_label), w.L, prm)
    full = ctx.label_loglik(*args).cpu().numpy()
    rng = np.random.default_rng(34)
    pix = rng.choice(w.N, 2990, replace=False).astype(np.int32)
    pix = np.concatenate([pix, [0, w.W - 1, w.N - w.W, w.N - 1], pix[:6]]).astype(np.int32)
    assert pix.size * 8 <= w.N
    got = ctx.label_loglik(*args, pix_subset=dev(pix)).cpu().numpy()
    assert np.array_equal(got.view(np.uint32), full[pix].view(np.uint32))
    small = pix[:600]
    got_s = ctx.label_loglik(*args, pix_subset=dev(small)).cpu().numpy()
    ref = oracle.label_loglik(w.rgb, masks, w.k, w.sample_pix, w.sample_label, w.L, alpha_rho=prm.alpha_rho,
                              sigma_c=prm.sigma_c, beta_scale=prm.beta_scale, rho_floor=prm.rho_floor_px,
                              pix=small)
    _ll_check(got_s, ref)


@pytest.mark.parametrize("levels", [0, 255])
def test_loglik_pixel_list_overflow_retry(ctx, levels):
    """The overflow-retry construction as a pixel list (every pixel three times
    in shuffled order): the overflowing sums are computed again on the
    matrix-core path, and each row equals the full-image row of its pixel bit
    for bit although its wave companions differ.  With colour levels the
    colours are 0 and 0.8 (distance 0.8 per channel)."""
    H, W = 16, 24
    rgb = np.full((3, H, W), 0.5 if levels == 0 else 0.0, np.float32)
    bad = [(r, c) for r in range(6, 10) for c in range(7, 17)]
    for r, c in bad:
        rgb[:, r, c] = 1.3 if levels == 0 else 204.0 / 255.0
    pixs = [r * W + c for r, c in bad]
    pixs[5] = 0
    pixs[15] = H * W - 1
    w = make_workload("retry_list", H=H, W=W, R=1, p=3, k=8, seed=1, per_region=2)
    w.rgb = rgb
    w.sample_pix = np.array(pixs, np.int32)
    w.sample_label = np.zeros(len(pixs), np.int32)
    w.L = 1
    w.k = 8
    w.colour_levels = levels
    masks = np.zeros((H * W, 1), np.uint64)
    pix = np.random.default_rng(4).permutation(np.tile(np.arange(H * W, dtype=np.int32), 3))
    got, ref = _loglik_both(ctx, w, masks, pix=pix)
    _ll_check(got, ref)
    st = ctx.last_loglik_stats()
    assert st["overflow_tiles"] > 0 and st["exact_tiles"] == 0, st
    full, _ = _loglik_both(ctx, w, masks)
    assert np.array_equal(got, full[pix])


@pytest.mark.parametrize("listed", [False, True], ids=["grid", "list"])
def test_loglik_exact_fixup_on_matrix_core_path(ctx, listed):
    """A spatial bandwidth so wide that the padding samples of the stream
    (parked 2^100 away) could reach the sum: every item is handed to the exact
    two-pass kernel, on the tile grid and on a pixel list."""
    w = _list_case()
    masks, _, _ = oracle.full_masks(w)
    pix = None
    if listed:
        pix = np.random.default_rng(8).integers(0, w.N, 1100).astype(np.int32)
    got, ref = _loglik_both(ctx, w, masks, pix=pix, rho_floor=1e10)
    _ll_check(got, ref)
    st = ctx.last_loglik_stats()
    assert st["exact_tiles"] > 0, st
