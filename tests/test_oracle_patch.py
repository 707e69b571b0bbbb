"""Pins of the oracle's patch analysis (gray value, patch, mask, normalisation,
analysed vector) against things other than the oracle itself."""
import os

import numpy as np
import pytest
from scipy.ndimage import correlate

import oracle
from workloads import make_workload

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _img(H=20, W=23, seed=3, R=3):
    return make_workload("t", H=H, W=W, R=R, p=5, k=12, seed=seed, per_region=5)


def test_mask_table_closed_form():
    # tests/golden/mask_p3.txt: closed form of the Sec. 3.1 Gaussian mask
    with open(os.path.join(GOLD, "mask_p3.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            p, sigma, vals = [c.strip() for c in line.split("|")]
            want = np.array([float(v) for v in vals.split()]).reshape(int(p), int(p))
            got = oracle.mask_table(int(p), float(sigma))
            np.testing.assert_allclose(got, want, rtol=2e-16, atol=0)


def _numpy_patches(rgb, p, sigma):
    """Independent brute force: numpy pad 'symmetric' (edge repeated),
    Gaussian mask, zero mean, unit norm."""
    r, g, b = [rgb[c].astype(np.float64) for c in range(3)]
    gray = (0.299 * r + 0.587 * g) + 0.114 * b
    h = p // 2
    pad = np.pad(gray, h, mode="symmetric")
    H, W = gray.shape
    u = np.arange(-h, h + 1)
    w = np.exp(-(u[:, None] ** 2 + u[None, :] ** 2) / (2 * sigma ** 2))
    out = np.empty((H * W, p * p))
    for row in range(H):
        for col in range(W):
            q = (pad[row:row + p, col:col + p] * w).ravel()
            z = q - q.mean()
            nrm = np.linalg.norm(z)
            out[row * W + col] = z / nrm if nrm > 0 else 0
    return out


@pytest.mark.parametrize("p", [3, 5, 7])
def test_patches_vs_numpy_bruteforce(p):
    w = _img()
    got = oracle.patches(w.rgb, p, p / 4.0)
    want = _numpy_patches(w.rgb, p, p / 4.0)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-13)


def test_patches_zero_mean_unit_norm():
    w = _img()
    s = oracle.patches(w.rgb, 7, 7 / 4.0)
    assert np.max(np.abs(s.sum(1))) < 1e-14
    assert np.max(np.abs(np.linalg.norm(s, axis=1) - 1)) < 1e-15


@pytest.mark.parametrize("p", [3, 5, 7, 11])
def test_analysis_as_filter_bank(p):
    """Sec. 5: the analysis is a bank of filters.  a_j(x) * nu(x) equals the
    correlation of the gray image with (O_j * mask) minus mu(x) * sum_t O_jt,
    computed here with scipy.ndimage.correlate (mode 'reflect' repeats the
    edge pixel, the same border rule)."""
    w = _img(H=24, W=27)
    k, n = 9, p * p
    rng = np.random.default_rng(p)
    om = rng.standard_normal((k, n)).astype(np.float32)
    sigma = p / 4.0
    alpha = oracle.analyze(w.rgb, p, sigma, om).reshape(24, 27, k)
    r, g, b = [w.rgb[c].astype(np.float64) for c in range(3)]
    gray = (0.299 * r + 0.587 * g) + 0.114 * b
    u = np.arange(-(p // 2), p // 2 + 1)
    mask = np.exp(-(u[:, None] ** 2 + u[None, :] ** 2) / (2 * sigma ** 2))
    mu = correlate(gray, mask, mode="reflect") / n
    nu2 = correlate(gray ** 2, mask ** 2, mode="reflect") - n * mu ** 2
    nu = np.sqrt(nu2)
    for j in range(k):
        K = om[j].astype(np.float64).reshape(p, p) * mask
        want = (correlate(gray, K, mode="reflect") - mu * om[j].astype(np.float64).sum()) / nu
        np.testing.assert_allclose(alpha[:, :, j], want, rtol=0, atol=1e-10)


def test_gain_invariance_bitwise():
    """Bias-and-gain model (Sec. 2): scaling the image by 2^e or by -1 leaves
    the normalised patch unchanged up to sign, so |a| and the co-supports are
    bit-identical."""
    w = _img()
    a0 = oracle.analyze(w.rgb, 5, 1.25, w.omega)
    for scale in (2.0 ** 5, 2.0 ** -7, -1.0, -0.25):
        a1 = oracle.analyze((w.rgb * np.float32(scale)).astype(np.float32), 5, 1.25, w.omega)
        assert np.array_equal(np.abs(a0), np.abs(a1))
    tau, _ = oracle.tau_median(a0, 0.1)
    m0 = oracle.cosupport(a0, tau)
    m1 = oracle.cosupport(oracle.analyze(-w.rgb, 5, 1.25, w.omega), tau)
    assert np.array_equal(m0, m1)


def test_gain_invariance_arbitrary_scale():
    w = _img()
    a0 = oracle.analyze(w.rgb, 5, 1.25, w.omega)
    tau, _ = oracle.tau_median(a0, 0.1)
    a1 = oracle.analyze((w.rgb.astype(np.float64) * 3.7).astype(np.float32), 5, 1.25, w.omega)
    # float32 rounding of the scaled image perturbs |a| slightly; masks agree
    # wherever |a| is not within that perturbation of tau
    m0 = np.abs(a0) <= tau
    m1 = np.abs(a1) <= tau
    near = np.abs(np.abs(a0) - tau) < 1e-5
    assert np.array_equal(m0[~near], m1[~near])
    assert np.max(np.abs(np.abs(a0) - np.abs(a1))) < 1e-5


def test_zero_patch_full_cosupport():
    """A zero patch has a = 0, so every index lies in the co-support (Sec. 2
    definition; zero-norm patches map to s = 0 by reading)."""
    rgb = np.zeros((3, 12, 13), dtype=np.float32)
    a = oracle.analyze(rgb, 5, 1.25, np.ones((70, 25), np.float32))
    assert np.all(a == 0)
    m = oracle.cosupport(a, 0.0)
    assert np.all(m[:, 0] == np.uint64(0xFFFFFFFFFFFFFFFF))
    assert np.all(m[:, 1] == np.uint64((1 << 6) - 1))  # padding bits stay 0


def test_nullspace_patch_lies_in_cosupport():
    """Sec. 2: a patch orthogonal to rows J of O has a_J = 0, so J is in its
    co-support.  The patch is built by projection: s orthogonal to O_J and to
    the constant vector; the gray values are chosen so that masking and
    normalisation return s (g_t = (c + s_t)/w_t)."""
    p, n, k = 5, 25, 40
    rng = np.random.default_rng(11)
    om = rng.standard_normal((k, n)).astype(np.float32)
    J = [1, 4, 7, 19, 33]
    A = np.vstack([om[J].astype(np.float64), np.ones((1, n))])
    v = rng.standard_normal(n)
    Q, _ = np.linalg.qr(A.T)
    s = v - Q @ (Q.T @ v)
    s /= np.linalg.norm(s)
    sigma = 1.25
    u = np.arange(-2, 3)
    w = np.exp(-(u[:, None] ** 2 + u[None, :] ** 2) / (2 * sigma ** 2)).ravel()
    g = ((3.0 + s) / w).reshape(5, 5)
    H = W = 9
    img = np.ones((H, W)) * 2.0
    img[2:7, 2:7] = g
    rgb = np.stack([img] * 3).astype(np.float32)
    a = oracle.analyze(rgb, p, sigma, om, pix=np.array([4 * W + 4], np.int32))[0]
    others = np.setdiff1d(np.arange(k), J)
    assert np.max(np.abs(a[J])) < 1e-5  # float32 image rounding only
    assert np.min(np.abs(a[others])) > 1e-4
    m = oracle.cosupport(a[None, :], 1e-5)[0]
    got = [j for j in range(k) if (int(m[j // 64]) >> (j % 64)) & 1]
    assert got == sorted(J)


def test_nonfinite_inputs_are_rejected(cfg0):
    """A NaN or an infinity in the colours or the operator has no meaning in the
    method (Sec. 2, Sec. 3.1): the oracle reports it instead of computing."""
    import numpy as np
    import oracle
    w = cfg0
    for which, val in (("rgb", np.nan), ("rgb", np.inf), ("omega", -np.inf)):
        rgb, om = w.rgb.copy(), w.omega.copy()
        (rgb if which == "rgb" else om).flat[17] = val
        with pytest.raises(oracle.OracleError) as e:
            oracle.analyze(rgb, w.p, w.mask_sigma, om)
        assert e.value.code == oracle.CSO_ERR_NONFINITE
    rgb = w.rgb.copy()
    rgb[1, 3, 4] = np.nan
    masks = np.zeros((w.N, 1), np.uint64)
    with pytest.raises(oracle.OracleError) as e:
        oracle.label_loglik(rgb, masks, w.k, w.sample_pix, w.sample_label, w.L)
    assert e.value.code == oracle.CSO_ERR_NONFINITE
