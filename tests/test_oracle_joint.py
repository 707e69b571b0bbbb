"""Pins of the oracle's joint data term (eq:joined): the colour/location Parzen
density of eq:color times the texture posterior of eq:post_text against each
label's textural representative (the majority definition of Sec. 2, the
median of eq:approx_cosupp for binary co-supports).  Checked against numpy's
median, Python sets, scipy's Gaussian densities and exact distance transform,
and against the invariants the posterior must satisfy."""
import numpy as np
import pytest
from scipy.ndimage import distance_transform_edt
from scipy.special import logsumexp
from scipy.stats import multivariate_normal

import oracle
from workloads import make_workload


@pytest.fixture(scope="module")
def small():
    w = make_workload("t", H=14, W=17, R=3, p=5, k=40, seed=21, per_region=6)
    masks, _, _ = oracle.full_masks(w)
    return w, masks


def _unpack(masks, k):
    """N x k array of 0/1 from N x ceil(k/64) words."""
    m = np.asarray(masks, dtype=np.uint64)
    j = np.arange(k)
    return ((m[:, j // 64] >> (j % 64).astype(np.uint64)) & np.uint64(1)).astype(np.int64)


def _bits(m, k):
    return {j for j in range(k) if (int(m[j // 64]) >> (j % 64)) & 1}


def test_rep_hand_cases():
    """Three samples 1100, 1010, 0110: bits 1..3 have two votes of three, bit 0
    none.  Two samples 01, 10: every bit is a tie, counted in."""
    masks = np.array([[0b1100], [0b1010], [0b0110], [0b01], [0b10]], np.uint64)
    pix = np.arange(5, dtype=np.int32)
    lab = np.array([0, 0, 0, 1, 1], np.int32)
    rep = oracle.label_rep(masks, 4, pix, lab, 2)
    assert rep[0, 0] == 0b1110
    assert rep[1, 0] == 0b0011


@pytest.mark.parametrize("k", [40, 64, 130])
def test_rep_is_componentwise_median(k):
    """c_i = component-wise median of the samples' 0/1 co-support vectors,
    with the middle value 1/2 of an even tie counted in."""
    rng = np.random.default_rng(5 + k)
    N, L = 300, 4
    words = (k + 63) // 64
    bits = (rng.random((N, k)) < 0.45).astype(np.uint64)
    masks = np.zeros((N, words), np.uint64)
    for j in range(k):
        masks[:, j // 64] |= bits[:, j] << np.uint64(j % 64)
    pix = rng.integers(0, N, 101).astype(np.int32)
    lab = rng.integers(0, L, 101).astype(np.int32)
    lab[:L] = np.arange(L)
    rep = oracle.label_rep(masks, k, pix, lab, L)
    got = _unpack(rep, k)
    for l in range(L):
        med = np.median(bits[pix[lab == l]].astype(np.float64), axis=0)
        assert np.array_equal(got[l], (med >= 0.5).astype(np.int64)), l


def _edt_d2(w, lab):
    seeds = np.zeros((w.H, w.W), dtype=bool)
    seeds.ravel()[w.sample_pix[w.sample_label == lab]] = True
    return np.rint(distance_transform_edt(~seeds) ** 2).astype(np.int64).ravel()


def _scipy_joint(w, masks, alpha_rho, sigma_c, beta_scale, rho_floor):
    """log of (1/m_i) sum_y N2(x; y, rho^2) N3(I(x); I(y), sigma_c^2), plus the
    log of softmax_i(-|Co_x xor c_i| / beta_i) with c_i from numpy's median."""
    N = w.H * w.W
    cols, rows = np.arange(N) % w.W, np.arange(N) // w.W
    rgb = w.rgb.reshape(3, N).astype(np.float64)
    onehot = _unpack(masks, w.k)
    sets = [_bits(masks[i], w.k) for i in range(N)]
    colour = np.empty((N, w.L))
    u = np.empty((N, w.L))
    for lab in range(w.L):
        ys = w.sample_pix[w.sample_label == lab]
        c = np.median(onehot[ys].astype(np.float64), axis=0) >= 0.5
        cset = {j for j in range(w.k) if c[j]}
        d2 = _edt_d2(w, lab)
        for x in range(N):
            rho = alpha_rho * np.sqrt(max(d2[x], rho_floor ** 2))
            z = np.array([cols[x], rows[x], *rgb[:, x]])
            Z = np.stack([cols[ys], rows[ys], *rgb[:, ys]], axis=1).astype(np.float64)
            cov = np.diag([rho ** 2] * 2 + [sigma_c ** 2] * 3)
            colour[x, lab] = logsumexp(multivariate_normal(mean=z, cov=cov).logpdf(Z)) - np.log(len(ys))
            u[x, lab] = -len(sets[x] ^ cset) / (beta_scale * rho)
    return colour + u - logsumexp(u, axis=1, keepdims=True)


@pytest.mark.parametrize("alpha_rho,sigma_c,beta_scale", [(1.3, 0.05, 1.0), (0.7, 0.2, 0.25)])
def test_joint_is_colour_kde_times_texture_posterior(small, alpha_rho, sigma_c, beta_scale):
    w, masks = small
    got = oracle.label_loglik(w.rgb, masks, w.k, w.sample_pix, w.sample_label, w.L,
                              alpha_rho=alpha_rho, sigma_c=sigma_c, beta_scale=beta_scale,
                              joint=True)
    want = _scipy_joint(w, masks, alpha_rho, sigma_c, beta_scale, 1.0)
    np.testing.assert_allclose(got, want, rtol=1e-11, atol=1e-10)


def test_texture_posterior_sums_to_one(small):
    """exp(joint - colour/location density) is a distribution over labels; the
    density is the per-sample form with the texture factor taken to 1."""
    w, masks = small
    joint = oracle.label_loglik(w.rgb, masks, w.k, w.sample_pix, w.sample_label, w.L, joint=True)
    colour = oracle.label_loglik(w.rgb, masks, w.k, w.sample_pix, w.sample_label, w.L,
                                 beta_scale=1e300)
    post = np.exp(joint - colour)
    np.testing.assert_allclose(post.sum(1), 1.0, rtol=0, atol=1e-12)
    assert (post > 0).all() and (post < 1).all()


def test_single_label_has_no_texture_term(small):
    w, masks = small
    one = np.zeros_like(w.sample_label)
    joint = oracle.label_loglik(w.rgb, masks, w.k, w.sample_pix, one, 1, joint=True)
    colour = oracle.label_loglik(w.rgb, masks, w.k, w.sample_pix, one, 1, beta_scale=1e300)
    np.testing.assert_allclose(joint, colour, rtol=0, atol=1e-12)


def test_equal_co_supports_give_uniform_posterior(small):
    """Every pixel with the same co-support: every TSM is 0, the posterior is 1/L."""
    w, masks = small
    same = np.repeat(masks[:1], masks.shape[0], axis=0)
    joint = oracle.label_loglik(w.rgb, same, w.k, w.sample_pix, w.sample_label, w.L, joint=True)
    colour = oracle.label_loglik(w.rgb, same, w.k, w.sample_pix, w.sample_label, w.L,
                                 beta_scale=1e300)
    np.testing.assert_allclose(joint, colour - np.log(w.L), rtol=0, atol=1e-12)


def test_nearer_representative_scores_higher():
    """One pixel, two labels at the same distance with the same colour: the
    label whose representative matches the pixel's co-support exactly gets
    posterior 1 / (1 + exp(-d / beta)) with d the other label's TSM."""
    H = W = 9
    rgb = np.full((3, H, W), 0.5, np.float32)
    k = 10
    masks = np.zeros((H * W, 1), np.uint64)
    x = 4 * W + 4
    ya, yb = 4 * W + 2, 4 * W + 6
    masks[x, 0] = masks[ya, 0] = 0b1111
    masks[yb, 0] = 0b1111110000  # TSM 10 to the pixel
    sp = np.array([ya, yb], np.int32)
    sl = np.array([0, 1], np.int32)
    px = np.array([x], np.int32)
    joint = oracle.label_loglik(rgb, masks, k, sp, sl, 2, pix=px, joint=True)[0]
    colour = oracle.label_loglik(rgb, masks, k, sp, sl, 2, pix=px, beta_scale=1e300)[0]
    beta = 1.3 * 2.0  # alpha_rho * distance 2, b = 1
    pa = 1.0 / (1.0 + np.exp(-10.0 / beta))
    np.testing.assert_allclose(np.exp(joint - colour), [pa, 1.0 - pa], rtol=1e-13)


def test_joint_normalised_and_subset(small):
    w, masks = small
    raw = oracle.label_loglik(w.rgb, masks, w.k, w.sample_pix, w.sample_label, w.L, joint=True)
    nrm = oracle.label_loglik(w.rgb, masks, w.k, w.sample_pix, w.sample_label, w.L, joint=True,
                              normalise=True)
    np.testing.assert_allclose(nrm, raw - logsumexp(raw, axis=1, keepdims=True), atol=1e-12)
    pix = np.array([3, 0, w.H * w.W - 1], np.int32)
    sub = oracle.label_loglik(w.rgb, masks, w.k, w.sample_pix, w.sample_label, w.L, pix=pix,
                              joint=True)
    assert np.array_equal(sub, raw[pix])


def test_joint_empty_label_is_an_error(small):
    w, masks = small
    with pytest.raises(oracle.OracleError) as e:
        oracle.label_loglik(w.rgb, masks, w.k, w.sample_pix, w.sample_label, w.L + 1, joint=True)
    assert e.value.code == oracle.CSO_ERR_EMPTY_LABEL
    with pytest.raises(oracle.OracleError):
        oracle.label_rep(masks, w.k, w.sample_pix, w.sample_label, w.L + 1)
