"""The allocation-free co-support call (cs_cosupport_noalloc) against the
allocating one (cs_cosupport), through the C-ABI: the same masks bit for bit,
on two calls in a row whose second input is smaller (the shared scratch keeps
the first call's contents), from stored analysed vectors and from the fused
analysis, in both precisions, at the proven and at an explicit margin; and
equal to the FP64 oracle's masks."""
import numpy as np
import pytest
import torch

import oracle
from workloads import make_workload

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.fixture(scope="module")
def ctx():
    from paper_1312_4746_amd import Context
    c = Context(0)
    yield c
    c.close()


CASES = [dict(name="big", H=96, W=131, R=4, p=11, k=242, seed=51),
         dict(name="small", H=21, W=30, R=3, p=5, k=50, seed=52)]


def _workload(c):
    c = dict(c)
    return make_workload(c.pop("name"), per_region=8, **c)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_noalloc_equals_cosupport_two_calls(ctx, prec):
    for case in CASES:  # the second call has the smaller input
        w = _workload(case)
        print(f"no-alloc case {case['name']} {prec}: {w.H}x{w.W} p={w.p} k={w.k}", flush=True)
        rgb, om = dev(w.rgb), dev(w.omega)
        a_ref = oracle.analyze(w.rgb, w.p, w.mask_sigma, w.omega)
        tau, _ = oracle.tau_median(a_ref, 0.1)
        m_ref = oracle.cosupport(a_ref, tau)
        alpha = ctx.analyze_patches(rgb, w.p, w.mask_sigma, om, precision=prec)
        for margin in (-1.0, 2.0 ** -8 * tau):
            for a in (alpha, None):
                want = ctx.cosupport(rgb, w.p, w.mask_sigma, om, tau, margin=margin, precision=prec, alpha=a)
                got = torch.full_like(want, -1)
                ctx.cosupport_noalloc(rgb, w.p, w.mask_sigma, om, tau, got, margin=margin, precision=prec,
                                      alpha=a)
                assert torch.equal(got, want), (case["name"], margin, a is None)
                if margin < 0:
                    assert np.array_equal(got.cpu().numpy().view(np.uint64), m_ref)


def test_noalloc_argument_errors(ctx):
    from paper_1312_4746_amd import CosparseError
    w = _workload(CASES[1])
    out = torch.empty((w.N, 1), dtype=torch.int64, device="cuda")
    with pytest.raises(CosparseError) as e:
        ctx.cosupport_noalloc(dev(w.rgb), w.p, w.mask_sigma, dev(w.omega), -1.0, out)
    assert e.value.code == 1
