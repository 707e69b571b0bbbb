"""Parity of the unsupervised data term (through the C-ABI) with the FP64
oracle (Sec. 3.1, unsupervised segmentation), and the unsupervised
segmentation with the label cost of eq:mdl.

Bars: k-medians classes and centroids bit for bit (integer popcounts and
counts); k-means classes equal wherever the oracle's nearest and second
nearest colour centroids differ by more than 1e-9 in squared distance (both
decide in FP64; the centroids differ only by the order of the FP64 sums), a
nearest centroid elsewhere, centroids within 1e-12; log-likelihoods within
1e-5 max(1, |l|) (FP32 output).
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import unsupervised as ou
from workloads import make_config, make_workload, unsup_init

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.fixture(scope="module")
def ctx():
    from paper_1312_4746_amd import Context
    c = Context(0)
    yield c
    c.close()


def _case(ctx, w, masks, Kc, Kt, iters, seed):
    from paper_1312_4746_amd import UnsupParams
    ic, it = unsup_init(w.N, Kc, Kt, seed)
    prm = UnsupParams(colour_classes=Kc, texture_classes=Kt, iterations=iters, sigma_c=0.05, beta=2.0)
    ll, info = ctx.unsupervised_loglik(dev(w.rgb), dev(masks.view(np.int64)), w.k, ic, it, prm)
    C, clab, _ = ou.kmeans_colour(w.rgb, ic, iters)
    T, tlab, _ = ou.kmedians_masks(masks, w.k, it, iters)
    # texture: exact
    assert np.array_equal(info["texture_labels"].cpu().numpy(), tlab)
    assert np.array_equal(info["texture_centroids"].cpu().numpy().view(np.uint64), T)
    # colour: FP64 decisions, sums in another order
    np.testing.assert_allclose(info["colour_centroids"].cpu().numpy(), C, atol=1e-12, rtol=0)
    X = w.rgb.reshape(3, -1).T.astype(np.float64)
    d = ((X[:, None] - C[None]) ** 2).sum(-1)
    srt = np.sort(d, 1)
    clear = (srt[:, 1] - srt[:, 0]) > 1e-9 if Kc > 1 else np.ones(w.N, bool)
    gl = info["colour_labels"].cpu().numpy()
    assert np.array_equal(gl[clear], clab[clear])
    assert np.all(d[np.arange(w.N), gl] <= srt[:, 0] + 1e-9)
    ref = ou.loglik(w.rgb, masks, w.k, C, T, 0.05, 2.0)
    got = ll.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(got - ref) <= 1e-5 * np.maximum(1.0, np.abs(ref))), float(np.abs(got - ref).max())
    return ll, info


@pytest.mark.parametrize("Kc,Kt,iters", [(4, 4, 10), (1, 3, 5), (3, 1, 0), (2, 16, 3), (16, 4, 6)])
def test_small_cases(ctx, Kc, Kt, iters):
    w = make_workload("us", H=41, W=67, R=4, p=5, k=70, seed=31, per_region=5)
    masks, _, _ = oracle.full_masks(w)
    _case(ctx, w, masks, Kc, Kt, iters, seed=Kc * 100 + Kt)


def test_bsds_shape(ctx):
    w = make_config(1)
    masks, _, _ = oracle.full_masks(w)
    _case(ctx, w, masks, 4, 4, 10, seed=7)


def test_unsupervised_segmentation_removes_labels(ctx):
    """The label cost of eq:mdl reduces the 16 initial classes; without it
    every class the data term favours somewhere survives."""
    from paper_1312_4746_amd import SegmentParams, UnsupParams
    w = make_config(1)
    rgb = dev(w.rgb)
    _, m, _ = ctx.cosupport_median(rgb, w.p, w.mask_sigma, dev(w.omega), 0.1)
    ic, it = unsup_init(w.N, 4, 4, 7)
    ll, _ = ctx.unsupervised_loglik(rgb, m, w.k, ic, it, UnsupParams(iterations=10))
    _, _, st0 = ctx.segment(rgb, ll, SegmentParams(lam=6.0, nu=0.0, iterations=300))
    _, _, st1 = ctx.segment(rgb, ll, SegmentParams(lam=6.0, nu=1100.0, iterations=300))
    assert st1["labels_used"] < st0["labels_used"] <= 16
    assert st1["binary"] >= st1["dual"]


def test_errors(ctx):
    from paper_1312_4746_amd import CosparseError, UnsupParams
    w = make_config(0)
    masks = dev(np.zeros((w.N, 1), np.int64))
    for prm, ic, it in ((UnsupParams(colour_classes=17), list(range(17)), [0, 1, 2, 3]),
                        (UnsupParams(beta=0.0), [0, 1, 2, 3], [0, 1, 2, 3]),
                        (UnsupParams(), [0, 1, 2, w.N], [0, 1, 2, 3])):
        with pytest.raises(CosparseError) as e:
            ctx.unsupervised_loglik(dev(w.rgb), masks, w.k, ic, it, prm)
        assert e.value.code == 1
