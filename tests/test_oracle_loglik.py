"""Pins of the oracle's per-pixel, per-label log-likelihood (Sec. 3.1 Parzen
sum with the co-support texture factor) against scipy's Gaussian densities,
scipy's exact distance transform, set-based TSM and invariants."""
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
    masks, tau, _ = oracle.full_masks(w)
    return w, masks


def _edt_d2(w, lab):
    seeds = np.zeros((w.H, w.W), dtype=bool)
    seeds.ravel()[w.sample_pix[w.sample_label == lab]] = True
    d = distance_transform_edt(~seeds)
    return np.rint(d ** 2).astype(np.int64).ravel()


def _bits(m, k):
    return {j for j in range(k) if (int(m[j // 64]) >> (j % 64)) & 1}


def test_nearest_d2_matches_scipy_edt(small):
    w, _ = small
    d2 = oracle.nearest_d2(w.H, w.W, w.sample_pix, w.sample_label, w.L)
    for lab in range(w.L):
        assert np.array_equal(d2[:, lab], _edt_d2(w, lab))


def _scipy_loglik(w, masks, alpha_rho, sigma_c, beta_scale, rho_floor):
    """log((1/m_i) sum_y N2(x; y, rho^2) N3(I(x); I(y), sigma_c^2) exp(-TSM/beta)),
    Gaussian log-densities from scipy.stats, TSM from Python sets, rho from
    scipy's exact distance transform."""
    N = w.H * w.W
    cols = np.arange(N) % w.W
    rows = np.arange(N) // w.W
    rgb = w.rgb.reshape(3, N).astype(np.float64)
    sets = [_bits(masks[i], w.k) for i in range(N)]
    out = np.empty((N, w.L))
    for lab in range(w.L):
        ys = w.sample_pix[w.sample_label == lab]
        d2 = _edt_d2(w, lab)
        for x in range(N):
            rho = alpha_rho * np.sqrt(max(d2[x], rho_floor ** 2))
            z = np.array([cols[x], rows[x], *rgb[:, x]])
            Z = np.stack([cols[ys], rows[ys], *rgb[:, ys]], axis=1).astype(np.float64)
            cov = np.diag([rho ** 2] * 2 + [sigma_c ** 2] * 3)
            lp = multivariate_normal(mean=z, cov=cov).logpdf(Z)
            tsm = np.array([len(sets[x] ^ sets[y]) for y in ys], dtype=np.float64)
            out[x, lab] = logsumexp(lp - tsm / (beta_scale * rho)) - np.log(len(ys))
    return out


def test_loglik_is_gaussian_kde_without_texture(small):
    """b -> infinity removes the texture factor; a floor larger than every
    distance makes rho constant: a textbook 5-D Gaussian KDE."""
    w, masks = small
    got = oracle.label_loglik(w.rgb, masks, w.k, w.sample_pix, w.sample_label, w.L,
                              alpha_rho=1.3, sigma_c=0.07, beta_scale=1e300, rho_floor=40.0)
    want = _scipy_loglik(w, masks, 1.3, 0.07, 1e300, 40.0)
    np.testing.assert_allclose(got, want, rtol=1e-11, atol=1e-11)


@pytest.mark.parametrize("alpha_rho,sigma_c,beta_scale", [(1.3, 0.05, 1.0), (0.7, 0.2, 3.0)])
def test_loglik_is_texture_weighted_kde(small, alpha_rho, sigma_c, beta_scale):
    w, masks = small
    got = oracle.label_loglik(w.rgb, masks, w.k, w.sample_pix, w.sample_label, w.L,
                              alpha_rho=alpha_rho, sigma_c=sigma_c, beta_scale=beta_scale,
                              rho_floor=1.0)
    want = _scipy_loglik(w, masks, alpha_rho, sigma_c, beta_scale, 1.0)
    np.testing.assert_allclose(got, want, rtol=1e-11, atol=1e-10)


def test_duplicated_samples_leave_loglik_unchanged(small):
    w, masks = small
    a = oracle.label_loglik(w.rgb, masks, w.k, w.sample_pix, w.sample_label, w.L)
    b = oracle.label_loglik(w.rgb, masks, w.k, np.concatenate([w.sample_pix, w.sample_pix]),
                            np.concatenate([w.sample_label, w.sample_label]), w.L)
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-12)


def test_permuted_samples_leave_loglik_unchanged(small):
    w, masks = small
    perm = np.random.default_rng(1).permutation(w.M)
    a = oracle.label_loglik(w.rgb, masks, w.k, w.sample_pix, w.sample_label, w.L)
    b = oracle.label_loglik(w.rgb, masks, w.k, w.sample_pix[perm], w.sample_label[perm], w.L)
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-12)


def test_normalised_form_sums_to_one(small):
    w, masks = small
    raw = oracle.label_loglik(w.rgb, masks, w.k, w.sample_pix, w.sample_label, w.L)
    nrm = oracle.label_loglik(w.rgb, masks, w.k, w.sample_pix, w.sample_label, w.L, normalise=True)
    np.testing.assert_allclose(np.exp(nrm).sum(1), 1.0, rtol=0, atol=1e-12)
    np.testing.assert_allclose(nrm, raw - logsumexp(raw, axis=1, keepdims=True), atol=1e-12)


def test_subset_rows_equal_full_rows(small):
    w, masks = small
    full = oracle.label_loglik(w.rgb, masks, w.k, w.sample_pix, w.sample_label, w.L)
    pix = np.array([0, 5, w.H * w.W - 1, 77], dtype=np.int32)
    sub = oracle.label_loglik(w.rgb, masks, w.k, w.sample_pix, w.sample_label, w.L, pix=pix)
    assert np.array_equal(sub, full[pix])


def test_empty_label_is_an_error(small):
    w, masks = small
    with pytest.raises(oracle.OracleError) as e:
        oracle.label_loglik(w.rgb, masks, w.k, w.sample_pix, w.sample_label, w.L + 1)
    assert e.value.code == oracle.CSO_ERR_EMPTY_LABEL


def test_closer_texture_scores_higher():
    """Two samples at the same distance with the same colour: the one whose
    co-support differs from the pixel's in fewer places contributes more, so
    removing it lowers the likelihood more than removing the other."""
    H = W = 9
    rgb = np.full((3, H, W), 0.5, np.float32)
    k = 10
    masks = np.zeros((H * W, 1), np.uint64)
    x = 4 * W + 4
    y_near_tex, y_far_tex = 4 * W + 2, 4 * W + 6
    masks[x, 0] = 0b1111
    masks[y_near_tex, 0] = 0b0111  # TSM 1
    masks[y_far_tex, 0] = 0b1111110000  # TSM 10
    both = oracle.label_loglik(rgb, masks, k, np.array([y_near_tex, y_far_tex], np.int32),
                               np.zeros(2, np.int32), 1, pix=np.array([x], np.int32))[0, 0]
    only_near = oracle.label_loglik(rgb, masks, k, np.array([y_near_tex, y_near_tex], np.int32),
                                    np.zeros(2, np.int32), 1, pix=np.array([x], np.int32))[0, 0]
    only_far = oracle.label_loglik(rgb, masks, k, np.array([y_far_tex, y_far_tex], np.int32),
                                   np.zeros(2, np.int32), 1, pix=np.array([x], np.int32))[0, 0]
    assert only_far < both < only_near
