"""Pins of the oracle's threshold, co-support masks and texture similarity."""
import itertools
import os

import numpy as np
import pytest

import oracle
from workloads import make_workload

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    with open(os.path.join(GOLD, name)) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            yield [c.strip() for c in line.split("|")]


def _mask_from_set(idx, k):
    m = np.zeros((k + 63) // 64, dtype=np.uint64)
    for j in idx:
        m[j // 64] |= np.uint64(1) << np.uint64(j % 64)
    return m


def _set_from_mask(m, k):
    return {j for j in range(k) if (int(m[j // 64]) >> (j % 64)) & 1}


def test_lower_median_golden():
    for frac, vals, med, tau in _rows("lower_median.txt"):
        a = np.array([float(v) for v in vals.split()])
        t, m = oracle.tau_median(a, float(frac))
        assert m == float(med)
        assert t == float(tau)


def test_tau_matches_numpy_partition():
    rng = np.random.default_rng(5)
    for cnt in (1, 2, 7, 1000, 1001):
        a = rng.standard_normal(cnt)
        t, m = oracle.tau_median(a, 0.1)
        r = (cnt - 1) // 2
        assert m == np.partition(np.abs(a), r)[r]
        assert t == 0.1 * m


def test_tsm_golden_hand_worked():
    for k, s1, s2, want in _rows("tsm_hand.txt"):
        k = int(k)
        A = [] if s1 == "-" else [int(v) for v in s1.split()]
        B = [] if s2 == "-" else [int(v) for v in s2.split()]
        got = oracle.tsm(_mask_from_set(A, k)[None], _mask_from_set(B, k)[None], k)[0, 0]
        assert got == int(want)


def test_tsm_sets_bruteforce_and_metric_axioms():
    rng = np.random.default_rng(9)
    for k in (5, 50, 64, 65, 98, 242):
        sets = [set(np.flatnonzero(rng.random(k) < q).tolist()) for q in (0.0, 0.05, 0.3, 0.5, 1.0)
                for _ in range(3)]
        M = np.stack([_mask_from_set(s, k) for s in sets])
        T = oracle.tsm(M, M, k)
        for i, j in itertools.product(range(len(sets)), repeat=2):
            a, b = sets[i], sets[j]
            assert T[i, j] == len(a) + len(b) - 2 * len(a & b) == len(a ^ b)
        assert np.array_equal(T, T.T)  # symmetric
        assert np.all(np.diag(T) == 0)  # identical patches: maximal similarity k - TSM = k
        assert T.min() >= 0 and T.max() <= k
        n = len(sets)
        for i, j, l in itertools.product(range(n), repeat=3):
            assert T[i, l] <= T[i, j] + T[j, l]  # Hamming metric


def test_tsm_of_negated_patch_is_zero():
    """s and -s have the same |a|, hence the same co-support: TSM = 0."""
    w = make_workload("t", H=16, W=18, R=2, p=5, k=40, seed=2, per_region=4)
    a = oracle.analyze(w.rgb, 5, 1.25, w.omega)
    tau, _ = oracle.tau_median(a, 0.1)
    m1 = oracle.cosupport(a, tau)
    m2 = oracle.cosupport(oracle.analyze(-w.rgb, 5, 1.25, w.omega), tau)
    T = oracle.tsm(m1, m2, 40)
    assert np.all(np.diag(T) == 0)


def test_cosupport_inclusive_threshold_and_padding():
    k = 70
    a = np.linspace(-1, 1, k)[None, :]
    tau = abs(a[0, 10])
    m = oracle.cosupport(a, tau)[0]
    got = _set_from_mask(m, k)
    assert got == {j for j in range(k) if abs(a[0, j]) <= tau}
    assert 10 in got  # |a_j| == tau is inside
    assert int(m[1]) >> (k - 64) == 0


def test_cosupport_fraction_matches_half_normal():
    """With a ~ N(0, 1/n) entries (Gaussian rows, unit-norm patches) and
    tau = 0.1 median|a|, about P(|Z| <= 0.1 * 0.6745) = 5.4 % of the bits are set."""
    w = make_workload("t", H=48, W=48, R=3, p=7, k=98, seed=4, per_region=10)
    masks, tau, alpha = oracle.full_masks(w)
    bits = sum(bin(int(v)).count("1") for v in masks.ravel())
    frac = bits / alpha.size
    assert 0.04 < frac < 0.07
    assert frac == pytest.approx(np.mean(np.abs(alpha) <= tau), abs=0)
