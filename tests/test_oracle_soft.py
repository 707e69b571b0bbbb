"""Pins of the oracle's joint data term with smooth co-supports (eq:map_tsm
iota(a) = exp(-a^2/sigma), the l1 texture distance of eq:tsm, the median
representative of eq:approx_cosupp, the posterior of eq:post_text): the
l1-centroid property of the median, the hard-co-support limit (which must
reproduce the pinned hard joint form), scipy densities, invariants."""
import numpy as np
import pytest
from scipy.ndimage import distance_transform_edt
from scipy.special import logsumexp
from scipy.stats import multivariate_normal

import oracle
from workloads import make_workload

SIGMA = 0.01


@pytest.fixture(scope="module")
def small():
    w = make_workload("t", H=14, W=17, R=3, p=5, k=40, seed=21, per_region=6)
    alpha = oracle.analyze(w.rgb, w.p, w.mask_sigma, w.omega)
    return w, alpha


def test_rep_is_an_l1_centroid(small):
    """Each c_lj minimises sum_s |c - iota_s| over the label's samples: no
    sample value and no small step either way does better, and it is one of
    the sample values (numpy's exp may differ from C's in the last place)."""
    w, alpha = small
    rep = oracle.label_rep_soft(alpha, SIGMA, w.sample_pix, w.sample_label, w.L)
    iota = np.exp(-alpha ** 2 / SIGMA)
    for l in range(w.L):
        v = iota[w.sample_pix[w.sample_label == l]]
        for j in range(w.k):
            f = lambda c: np.abs(c - v[:, j]).sum()  # noqa: E731
            c = rep[l, j]
            assert np.isclose(v[:, j], c, rtol=4e-16, atol=0).any()  # a sample's value (its exp)
            best = min(f(x) for x in v[:, j])
            assert f(c) <= best + 1e-14
            assert f(c) <= f(c + 1e-9) + 1e-14 and f(c) <= f(c - 1e-9) + 1e-14


def test_rep_even_count_takes_the_upper_middle():
    """Two samples per label: the larger of the two values (rank floor(m/2))."""
    alpha = np.array([[0.0, 0.3], [0.2, 0.0], [0.05, 0.05], [0.5, 0.1]])
    sp = np.arange(4, dtype=np.int32)
    sl = np.array([0, 0, 1, 1], np.int32)
    rep = oracle.label_rep_soft(alpha, SIGMA, sp, sl, 2)
    io = np.exp(-alpha ** 2 / SIGMA)
    np.testing.assert_array_equal(rep[0], np.maximum(io[0], io[1]))
    np.testing.assert_array_equal(rep[1], np.maximum(io[2], io[3]))


def test_hard_limit_reproduces_the_hard_joint_form(small):
    """Analysed entries that are exactly 0 or at least 1 in magnitude: iota is
    1 or below e^-100, the smooth co-support is the hard one at tau = 0, and
    the soft form equals the hard joint form with masks [a_j = 0] (majority
    with ties in = upper median of 0/1 values; l1 distance = TSM)."""
    w, _ = small
    rng = np.random.default_rng(8)
    N = w.H * w.W
    zero = rng.random((N, w.k)) < 0.5
    alpha = np.where(zero, 0.0, rng.choice([-1.0, 1.0], (N, w.k)) * (1.0 + rng.random((N, w.k))))
    masks = np.zeros((N, 1), np.uint64)
    for j in range(w.k):
        masks[:, 0] |= zero[:, j].astype(np.uint64) << np.uint64(j)
    soft = oracle.label_loglik_soft(w.rgb, alpha, SIGMA, w.sample_pix, w.sample_label, w.L)
    hard = oracle.label_loglik(w.rgb, masks, w.k, w.sample_pix, w.sample_label, w.L, joint=True)
    np.testing.assert_allclose(soft, hard, rtol=1e-12, atol=1e-12)


def _edt_d2(w, lab):
    seeds = np.zeros((w.H, w.W), dtype=bool)
    seeds.ravel()[w.sample_pix[w.sample_label == lab]] = True
    return np.rint(distance_transform_edt(~seeds) ** 2).astype(np.int64).ravel()


def test_soft_is_colour_kde_times_l1_posterior(small):
    """scipy's 5-D Gaussian KDE plus the log-softmax of -||c_i - iota(a_x)||_1 / beta_i
    with c_i from numpy's sort and rho from scipy's distance transform."""
    w, alpha = small
    got = oracle.label_loglik_soft(w.rgb, alpha, SIGMA, w.sample_pix, w.sample_label, w.L,
                                   sigma_c=0.07, beta_scale=0.5)
    N = w.H * w.W
    cols, rows = np.arange(N) % w.W, np.arange(N) // w.W
    rgb = w.rgb.reshape(3, N).astype(np.float64)
    iota = np.exp(-alpha ** 2 / SIGMA)
    colour = np.empty((N, w.L))
    u = np.empty((N, w.L))
    for lab in range(w.L):
        ys = w.sample_pix[w.sample_label == lab]
        c = np.sort(iota[ys], axis=0)[len(ys) // 2]
        d2 = _edt_d2(w, lab)
        for x in range(N):
            rho = 1.3 * np.sqrt(max(d2[x], 1.0))
            z = np.array([cols[x], rows[x], *rgb[:, x]])
            Z = np.stack([cols[ys], rows[ys], *rgb[:, ys]], axis=1).astype(np.float64)
            cov = np.diag([rho ** 2] * 2 + [0.07 ** 2] * 3)
            colour[x, lab] = logsumexp(multivariate_normal(mean=z, cov=cov).logpdf(Z)) - np.log(len(ys))
            u[x, lab] = -np.abs(c - iota[x]).sum() / (0.5 * rho)
    want = colour + u - logsumexp(u, axis=1, keepdims=True)
    np.testing.assert_allclose(got, want, rtol=1e-11, atol=1e-10)


def test_soft_posterior_sums_to_one_and_wide_sigma_is_uniform(small):
    w, alpha = small
    masks = oracle.cosupport(alpha, 0.0)
    colour = oracle.label_loglik(w.rgb, masks, w.k, w.sample_pix, w.sample_label, w.L,
                                 beta_scale=1e300)
    soft = oracle.label_loglik_soft(w.rgb, alpha, SIGMA, w.sample_pix, w.sample_label, w.L)
    np.testing.assert_allclose(np.exp(soft - colour).sum(1), 1.0, rtol=0, atol=1e-12)
    wide = oracle.label_loglik_soft(w.rgb, alpha, 1e300, w.sample_pix, w.sample_label, w.L)
    np.testing.assert_allclose(wide, colour - np.log(w.L), rtol=0, atol=1e-12)


def test_soft_normalised_subset_and_errors(small):
    w, alpha = small
    raw = oracle.label_loglik_soft(w.rgb, alpha, SIGMA, w.sample_pix, w.sample_label, w.L)
    nrm = oracle.label_loglik_soft(w.rgb, alpha, SIGMA, w.sample_pix, w.sample_label, w.L,
                                   normalise=True)
    np.testing.assert_allclose(nrm, raw - logsumexp(raw, axis=1, keepdims=True), atol=1e-12)
    pix = np.array([5, 0, w.H * w.W - 1], np.int32)
    sub = oracle.label_loglik_soft(w.rgb, alpha, SIGMA, w.sample_pix, w.sample_label, w.L, pix=pix)
    assert np.array_equal(sub, raw[pix])
    with pytest.raises(oracle.OracleError) as e:
        oracle.label_loglik_soft(w.rgb, alpha, SIGMA, w.sample_pix, w.sample_label, w.L + 1)
    assert e.value.code == oracle.CSO_ERR_EMPTY_LABEL
    with pytest.raises(oracle.OracleError) as e:
        oracle.label_loglik_soft(w.rgb, alpha, 0.0, w.sample_pix, w.sample_label, w.L)
    assert e.value.code == oracle.CSO_ERR_ARG
