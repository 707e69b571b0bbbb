"""FP64 oracle of the unsupervised data term (paper Sec. 3.1, "Unsupervised
Segmentation"; Sec. 3.2, eq:mdl).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark may import this module; the product library never does.

With no scribbles the segment classes are found by clustering:

* colour classes: k-means on the pixels' colours (Lloyd's iteration: assign
  every pixel to its nearest centroid in squared Euclidean distance, then
  move every centroid to the mean of its pixels);
* texture classes: k-medians on the pixels' co-supports (assign by the
  texture similarity TSM, the Hamming distance of the masks; the centroid
  of a class is its component-wise median, i.e. the majority of its masks);
* segment classes: every pair (colour class a, texture class b), class index
  i = a K_t + b, represented by the two centroids;
* per pixel a colour and a texture likelihood in the form of eq:post_text
  (an exponential of minus a distance, normalised over the classes), their
  product the joint likelihood of eq:joined, f_i = -log of it the data term.

Readings (also in the design notes): the initial centroids are the colours
and masks of caller-given pixels (random numbers of the method are inputs);
a fixed number of iterations; distance ties go to the lowest class; a class
left without pixels keeps its centroid; a majority tie (exactly half of the
masks) puts the component in the median, as for the hard representatives;
the colour distance is ||I(x) - mu_a||^2 / (2 sigma_c^2) (the Gaussian kernel
of eq:color) and the texture distance TSM(x, c_b) / beta with a constant beta
(no scribbles, so no location-dependent bandwidth).
"""
from __future__ import annotations

import numpy as np


def popcount64(a: np.ndarray) -> np.ndarray:
    """Bits set in each uint64."""
    a = np.ascontiguousarray(a, dtype=np.uint64)
    return np.unpackbits(a.view(np.uint8).reshape(*a.shape, 8), axis=-1).sum(-1)


def kmeans_colour(rgb: np.ndarray, init_pix, iterations: int):
    """Lloyd's k-means on the colours of every pixel: `iterations` times
    assign and update, then assign to the final centroids.  Returns
    (centroids (K, 3) FP64, labels (N,) int32, objective of each assignment)."""
    X = np.asarray(rgb, np.float64).reshape(3, -1).T
    C = X[np.asarray(init_pix, np.int64)].copy()

    def assign(C):
        d = ((X[:, None, :] - C[None, :, :]) ** 2).sum(-1)
        lab = np.argmin(d, axis=1).astype(np.int32)  # ties: lowest class
        return lab, float(d[np.arange(X.shape[0]), lab].sum())

    hist = []
    for _ in range(iterations):
        lab, obj = assign(C)
        hist.append(obj)
        for a in range(C.shape[0]):
            sel = lab == a
            if sel.any():  # a class without pixels keeps its centroid
                C[a] = X[sel].sum(0) / sel.sum()
    lab, obj = assign(C)
    hist.append(obj)
    return C, lab, np.asarray(hist)


def mask_bits(masks: np.ndarray, k: int) -> np.ndarray:
    """(N, words) uint64 masks as (N, k) 0/1 integers, bit j of word j/64 at column j."""
    M = np.ascontiguousarray(masks, np.uint64)
    N, nw = M.shape
    return np.unpackbits(M.view(np.uint8).reshape(N, nw * 8), axis=1, bitorder="little")[:, :k].astype(np.int64)


def pack_bits(bits: np.ndarray) -> np.ndarray:
    """(K, k) 0/1 integers as (K, ceil(k/64)) uint64 masks."""
    K, k = bits.shape
    out = np.zeros((K, (k + 63) // 64), np.uint64)
    for j in range(k):
        out[:, j // 64] |= bits[:, j].astype(np.uint64) << np.uint64(j % 64)
    return out


def kmedians_masks(masks: np.ndarray, k: int, init_pix, iterations: int):
    """k-medians on the co-support masks (N, ceil(k/64)) uint64 with the
    Hamming distance (TSM): `iterations` times assign and update, then
    assign.  Returns (centroids (K, words) uint64, labels (N,) int32,
    objective of each assignment)."""
    bits = mask_bits(masks, k)
    N = bits.shape[0]
    C = bits[np.asarray(init_pix, np.int64)].copy()

    def assign(C):
        d = np.stack([(bits != C[b][None]).sum(1) for b in range(C.shape[0])], 1)
        lab = np.argmin(d, axis=1).astype(np.int32)
        return lab, int(d[np.arange(N), lab].sum())

    hist = []
    for _ in range(iterations):
        lab, obj = assign(C)
        hist.append(obj)
        for b in range(C.shape[0]):
            sel = lab == b
            n = int(sel.sum())
            if n:  # component-wise median of 0/1 values: the majority, a tie in
                C[b] = (2 * bits[sel].sum(0) >= n).astype(np.int64)
    lab, obj = assign(C)
    hist.append(obj)
    return pack_bits(C), lab, np.asarray(hist)


def loglik(rgb: np.ndarray, masks: np.ndarray, k: int, ccent: np.ndarray, tcent: np.ndarray, sigma_c: float,
           beta: float) -> np.ndarray:
    """Per-pixel log-likelihood of every segment class i = a K_t + b:
    log P(I(x) | a) + log P(s_x | b), each an exponential of minus the
    distance normalised over all K_c K_t classes (eq:post_text form)."""
    X = np.asarray(rgb, np.float64).reshape(3, -1).T
    Kc, Kt = ccent.shape[0], tcent.shape[0]
    dc = ((X[:, None, :] - np.asarray(ccent, np.float64)[None]) ** 2).sum(-1) / (2.0 * sigma_c * sigma_c)
    M = np.ascontiguousarray(masks, np.uint64)
    dt = np.stack([popcount64(M ^ tcent[b][None]).sum(1) for b in range(Kt)], 1).astype(np.float64) / beta
    # exponent of every class, then normalised over all classes
    ec = -np.repeat(dc, Kt, axis=1)   # class a * Kt + b -> colour class a
    et = -np.tile(dt, (1, Kc))        # -> texture class b
    def lnorm(e):
        m = e.max(1, keepdims=True)
        return e - (m + np.log(np.exp(e - m).sum(1, keepdims=True)))
    return lnorm(ec) + lnorm(et)
