"""Pins of the FP64 oracle of the unsupervised data term (Sec. 3.1): k-means
against scikit-learn's Lloyd iteration from the same start, the descent of
both clustering objectives, the k-medians centroid as numpy's component-wise
median and as the brute-force minimiser of the summed Hamming distance, and
the class likelihoods as log-softmaxes (scipy) of the two distances."""
import itertools

import numpy as np
import pytest
from scipy.special import log_softmax

from oracle import unsupervised as ou


def _blobs(rng, centres, n_each, sd=0.03):
    pts = np.concatenate([c + rng.normal(0, sd, (n_each, 3)) for c in centres])
    return pts.T.reshape(3, 1, -1).astype(np.float32)


def test_kmeans_matches_scikit_learn_lloyd():
    from sklearn.cluster import KMeans
    rng = np.random.default_rng(1)
    centres = [np.array([0.1, 0.2, 0.3]), np.array([0.8, 0.1, 0.5]), np.array([0.4, 0.9, 0.2])]
    rgb = _blobs(rng, centres, 200)
    init = np.array([5, 250, 590])
    C, lab, hist = ou.kmeans_colour(rgb, init, 30)
    X = rgb.reshape(3, -1).T.astype(np.float64)
    km = KMeans(n_clusters=3, init=X[init], n_init=1, max_iter=30, tol=0.0, algorithm="lloyd").fit(X)
    np.testing.assert_allclose(C, km.cluster_centers_, atol=1e-12)
    assert np.array_equal(lab, km.labels_)


def test_kmeans_objective_descends_and_fixed_point():
    rng = np.random.default_rng(2)
    rgb = rng.uniform(0, 1, (3, 20, 30)).astype(np.float32)
    C, lab, hist = ou.kmeans_colour(rgb, rng.choice(600, 5, replace=False), 25)
    assert np.all(np.diff(hist) <= 1e-12)
    X = rgb.reshape(3, -1).T.astype(np.float64)
    for a in range(5):
        if (lab == a).any():
            np.testing.assert_allclose(C[a], X[lab == a].mean(0), atol=1e-9)
    d = ((X[:, None] - C[None]) ** 2).sum(-1)
    assert np.all(d[np.arange(600), lab] <= d.min(1) + 1e-15)


@pytest.mark.parametrize("k", [6, 70])
def test_kmedians_centroid_is_the_median_and_minimises_hamming(k):
    rng = np.random.default_rng(k)
    nw = (k + 63) // 64
    M = rng.integers(0, 2 ** 63, size=(300, nw), dtype=np.int64).view(np.uint64)
    if k % 64:
        M[:, -1] &= np.uint64((1 << (k % 64)) - 1)
    C, lab, hist = ou.kmedians_masks(M, k, rng.choice(300, 4, replace=False), 8)
    assert np.all(np.diff(hist) <= 0)
    bits = ou.mask_bits(M, k)
    cb = ou.mask_bits(C, k)
    # the last centroids are the medians of the assignment before them: check
    # the fixed-point form on a converged run instead
    C2, lab2, _ = ou.kmedians_masks(M, k, rng.choice(300, 4, replace=False), 40)
    cb2 = ou.mask_bits(C2, k)
    for b in range(4):
        sel = lab2 == b
        if not sel.any():
            continue
        med = (np.median(bits[sel], axis=0) >= 0.5).astype(np.int64)  # a tie (0.5) is in
        assert np.array_equal(cb2[b], med)
        if k <= 8:
            costs = {cand: int((bits[sel] != np.array(cand)).sum()) for cand in itertools.product((0, 1), repeat=k)}
            assert costs[tuple(cb2[b])] == min(costs.values())
    assert cb.shape == (4, k)


def test_kmedians_tie_goes_in():
    M = np.array([[0b01], [0b11]], dtype=np.uint64)  # two masks, bit 1 set in one of them
    C, lab, _ = ou.kmedians_masks(M, 2, [0], 1)
    assert int(C[0, 0]) == 0b11


def test_class_likelihoods_are_two_log_softmaxes():
    rng = np.random.default_rng(5)
    rgb = rng.uniform(0, 1, (3, 6, 7)).astype(np.float32)
    k = 90
    M = rng.integers(0, 2 ** 63, size=(42, 2), dtype=np.int64).view(np.uint64)
    M[:, 1] &= np.uint64((1 << 26) - 1)
    cc = rng.uniform(0, 1, (3, 3))
    tc = M[[0, 7, 30, 41]]
    ll = ou.loglik(rgb, M, k, cc, tc, 0.1, 2.5)
    X = rgb.reshape(3, -1).T.astype(np.float64)
    dc = ((X[:, None] - cc[None]) ** 2).sum(-1) / (2 * 0.01)
    dt = np.array([[bin(int(a) ^ int(b)).count("1") + bin(int(c) ^ int(d)).count("1")
                    for (b, d) in tc] for (a, c) in M], np.float64) / 2.5
    ref = np.zeros((42, 12))
    for a in range(3):
        for b in range(4):
            ref[:, a * 4 + b] = (log_softmax(-dc, axis=1)[:, a] - np.log(4)) + (log_softmax(-dt, axis=1)[:, b] - np.log(3))
    np.testing.assert_allclose(ll, ref, atol=1e-12)
    # the most likely class pairs the nearest colour and texture centroids
    best = np.argmax(ll, 1)
    assert np.array_equal(best // 4, np.argmin(dc, 1))
    assert np.array_equal(best % 4, np.argmin(dt, 1))
