"""Status codes and state of the context through the C-ABI: the optional
finite check of the inputs, and the log-likelihood counters, which live in
context-owned device memory and survive other calls."""
import numpy as np
import pytest
import torch

import oracle
from workloads import make_config, make_workload

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.fixture(scope="module")
def ctx():
    from paper_1312_4746_amd import Context
    c = Context(0)
    yield c
    c.close()


def test_nonfinite_inputs_rejected_when_checked(ctx):
    from paper_1312_4746_amd import CosparseError, LoglikParams
    from paper_1312_4746_amd.binding import CS_ERR_NONFINITE
    w = make_config(0)
    bad_rgb = w.rgb.copy()
    bad_rgb[2, 5, 7] = np.nan
    bad_om = w.omega.copy()
    bad_om[3, 4] = np.inf
    masks, _, _ = oracle.full_masks(w)
    ctx.set_check_finite(True)
    try:
        for rgb, om in ((bad_rgb, w.omega), (w.rgb, bad_om)):
            with pytest.raises(CosparseError) as e:
                ctx.analyze_patches(dev(rgb), w.p, w.mask_sigma, dev(om))
            assert e.value.code == CS_ERR_NONFINITE
            with pytest.raises(CosparseError) as e:
                ctx.cosupport_median(dev(rgb), w.p, w.mask_sigma, dev(om), 0.1)
            assert e.value.code == CS_ERR_NONFINITE
            with pytest.raises(CosparseError) as e:
                ctx.cosupport(dev(rgb), w.p, w.mask_sigma, dev(om), 0.01)
            assert e.value.code == CS_ERR_NONFINITE
        with pytest.raises(CosparseError) as e:
            ctx.label_loglik(dev(bad_rgb), dev(masks.view(np.int64)), w.k, dev(w.sample_pix),
                             dev(w.sample_label), w.L, LoglikParams())
        assert e.value.code == CS_ERR_NONFINITE
        # finite inputs pass the check and give the oracle's results
        a = ctx.analyze_patches(dev(w.rgb), w.p, w.mask_sigma, dev(w.omega))
        tau = ctx.tau_median(dev(w.rgb), w.p, w.mask_sigma, dev(w.omega), a, 0.1)
        assert tau == oracle.tau_median(oracle.analyze(w.rgb, w.p, w.mask_sigma, w.omega), 0.1)[0]
    finally:
        ctx.set_check_finite(False)
    # off: no check, no error (the output is unspecified)
    ctx.analyze_patches(dev(bad_rgb), w.p, w.mask_sigma, dev(w.omega))
    torch.cuda.synchronize()


def test_loglik_counters_survive_other_calls(ctx):
    """The counters of a log-likelihood call stay readable after co-support,
    analysis and surrogate calls that carve the same workspace."""
    from paper_1312_4746_amd import LoglikParams, Mlp
    from workloads import mlp_init
    b = make_config(1)  # the BSDS-sized case rescales a few thousand wave-chunks
    brgb = dev(b.rgb)
    _, bm, _ = ctx.cosupport_median(brgb, b.p, b.mask_sigma, dev(b.omega), 0.1)
    prm = LoglikParams(alpha_rho=b.alpha_rho, sigma_c=b.sigma_c, beta_scale=b.beta_scale,
                       rho_floor_px=b.rho_floor_px, colour_levels=b.colour_levels)
    ctx.label_loglik(brgb, bm, b.k, dev(b.sample_pix), dev(b.sample_label), b.L, prm)
    first = ctx.last_loglik_stats()
    assert first["rescaled_chunks"] > 0
    w = make_workload("st", H=40, W=56, R=3, p=5, k=40, seed=21, per_region=20)
    alpha, m, _ = ctx.cosupport_median(dev(w.rgb), w.p, w.mask_sigma, dev(w.omega), 0.1)
    ctx.tau_median(dev(w.rgb), w.p, w.mask_sigma, dev(w.omega), alpha, 0.1, precision="bf16")
    net = Mlp(ctx, 20, 3, dev(mlp_init(20, 128, 3, 1)))
    x = torch.randn(4096, 20, device="cuda")
    net.grad(x, torch.randn(4096, 3, device="cuda"))
    net.close()
    assert ctx.last_loglik_stats() == first
    # a subset call resets them to zero (no full-image counters)
    ctx.label_loglik(brgb, bm, b.k, dev(b.sample_pix), dev(b.sample_label), b.L, prm,
                     pix_subset=dev(np.arange(10, dtype=np.int32)))
    assert ctx.last_loglik_stats() == {"rescaled_chunks": 0, "overflow_tiles": 0, "exact_tiles": 0}
