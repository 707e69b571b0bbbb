"""Benchmark of the co-sparse data term on one MI355X.

One step = the whole data-term path over one synthetic image: analysed
vectors (MFMA), exact threshold tau, co-support masks, and the per-pixel,
per-label log-likelihood (distance transform + Parzen sum).  The default
workload is the large case: 1024x1024 RGB, 11x11 patches, k = 242, 16 labels,
50,000 scribble samples, FP32 (5.24e10 pixel x sample pairs per step).
Inputs are resident in HBM before timing starts.

Prints one JSON line with the whole-job throughput (pixel x sample pairs/s),
the roofline of the dominant kernel (the Parzen sum, measured with HIP events
on the stream it runs on), the FP64 oracle timed on the host on a bounded
sample of the same workload, and the learned surrogate's pixel rate on its
own workload (2048x2048) with its flip rate against the exact path.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks: FP32 vector 157.3 TFLOP/s (256 CUs x 4 SIMDs x 16
# lanes x 2.4 GHz x 2 flops per FMA x 2 for packed FP32), FP32 matrix 157.3
# TFLOP/s, BF16 dense matrix 2.5 PFLOP/s, HBM3E 8 TB/s.
PEAK_FP32_VECTOR = 157.3e12
PEAK_HBM = 8.0e12
PEAK_MFMA = {"fp32": 157.3e12, "bf16": 2.5e15}
# issue model of the VALU (measured on gfx950 with a probe kernel): a wave64
# VALU instruction occupies its SIMD for 4 cycles, a transcendental for 8
SIMDS, CLOCK_HZ, VALU_CYCLES, TRANS_CYCLES = 1024, 2.4e9, 4, 8
# the Parzen kernel carries timing events on one launch in this many inside the timed region
PARZEN_EVENT_PERIOD = 8
# smooth co-support map exp(-a^2 / sigma) of the paper's experiments
SIGMA_IOTA = 0.01


def parzen_ops_per_pair(k: int, texture: bool = True) -> int:
    """Algorithmic VALU issue slots per pixel x sample pair of the direct
    evaluation: location difference and square (4), colour differences and
    squares (6), XOR and popcount per 32-bit co-support word (2 ceil(k/32)),
    conversion of the count and the three-term exponent (4), log-sum-exp
    max, shift and accumulate (3), and one v_exp_f32 at a quarter of the
    FP32 issue rate (4 slots).  Without the texture factor in the sum (the
    joint forms): no popcounts, no conversion, a two-term exponent (2)."""
    if not texture:
        return 4 + 6 + 2 + 3 + 4
    return 17 + 2 * ((k + 31) // 32) + 4


def load_profile(name: str):
    """A committed counter summary (profiles/<name>) or None."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            return json.load(f)
    except Exception:
        return None


def kernel_source_digest() -> str:
    """Digest of the Parzen kernel's source, of its argument struct and of the
    host code that cuts its work order into label blocks (the counters stay
    valid while none of them changes)."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_1312_4746_amd", "csrc")
    h = hashlib.sha256()
    with open(os.path.join(csrc, "k_parzen_mfma.hip"), "rb") as fh:
        h.update(fh.read())
    with open(os.path.join(csrc, "cs_internal.h")) as fh:
        hdr = fh.read()
    a = hdr.index("struct ParzenFastArgs")
    h.update(hdr[a:hdr.index("};", a)].encode())
    with open(os.path.join(csrc, "cs_host.hip")) as fh:
        host = fh.read()
    a = host.index("// labels per block of the work order")
    h.update(host[a:host.index("fa.lblock = lb;", a)].encode())
    return h.hexdigest()[:16]


def precision_sweep(ctx, w, rgb, om, alpha, spix, slab, prm):
    """BF16 analysis with FP64 recompute inside a margin of tau: co-support
    bits that differ from the exact masks (those of the proven margin, which
    equal the FP64 masks bit for bit), the entries recomputed, and the effect
    of the differing bits on the log-likelihoods."""
    import numpy as np
    import torch
    tau = ctx.tau_median(rgb, w.p, w.mask_sigma, om, alpha, w.tau_frac, precision="bf16")
    exact, st = ctx.cosupport(rgb, w.p, w.mask_sigma, om, tau, precision="bf16", alpha=alpha, stats=True)
    ll_exact = ctx.label_loglik(rgb, exact, w.k, spix, slab, w.L, prm)
    rows = []
    for name, margin in (("2^-8 tau", 2.0 ** -8 * tau), ("2^-6 tau", 2.0 ** -6 * tau),
                         ("2^-4 tau", 2.0 ** -4 * tau), ("proven bound", -1.0)):
        m, s = ctx.cosupport(rgb, w.p, w.mask_sigma, om, tau, margin=margin, precision="bf16", alpha=alpha,
                             stats=True)
        x = torch.bitwise_xor(m, exact)
        bits = int(np.unpackbits(x.cpu().numpy().view(np.uint8)).sum())
        ll = ctx.label_loglik(rgb, m, w.k, spix, slab, w.L, prm)
        d = (ll - ll_exact).abs()
        rows.append({"margin": name, "margin_value": (margin if margin >= 0 else s["max_margin"]),
                     "mismatched_bits": bits, "recomputed": s["recomputed"],
                     "recompute_fraction": s["recomputed"] / float(w.N * w.k),
                     "max_abs_dl_vs_exact_masks": float(d.max()), "mean_abs_dl": float(d.mean())})
    return {"tau": tau, "proven_margin_max": st["max_margin"], "rows": rows}


def cpu_baseline(w, n_sample: int, joint: bool = False, soft: bool = False, n_front: int = 65536):
    """The FP64 oracle on the host, on a bounded sample of the workload: the
    Parzen log-likelihood of n_sample evenly strided pixels, plus their share
    of the front end (analysis, tau and masks of every pixel, needed for any
    pixel).  Up to 2 n_front pixels the front end runs on the whole image;
    above, it runs on n_front strided pixels and is scaled to the image:
    analysis and masks by the pixel count, the sort of the median by
    n log n of the entry count (an extrapolation, stated in the sample)."""
    import math

    import numpy as np

    import oracle
    oracle.lib()
    N, k = w.N, w.k
    nw = (k + 63) // 64
    pix = np.linspace(0, N - 1, n_sample).astype(np.int32)
    if N <= 2 * n_front:
        t0 = time.perf_counter()
        alpha = oracle.analyze(w.rgb, w.p, w.mask_sigma, w.omega)
        if not soft:  # the smooth form needs no threshold and no masks
            tau, _ = oracle.tau_median(alpha, w.tau_frac)
            masks = oracle.cosupport(alpha, tau)
        t_front = time.perf_counter() - t0
        how = f"analysis{'' if soft else ', tau and masks'} of all {N} pixels ({t_front:.2f} s)"
    else:
        fpix = np.linspace(0, N - 1, n_front).astype(np.int32)
        t0 = time.perf_counter()
        a_f = oracle.analyze(w.rgb, w.p, w.mask_sigma, w.omega, pix=fpix)
        t_an = time.perf_counter() - t0
        tau = None
        t_sort = t_cos = 0.0
        if not soft:
            t0 = time.perf_counter()
            tau, _ = oracle.tau_median(a_f, w.tau_frac)
            t_sort = time.perf_counter() - t0
            t0 = time.perf_counter()
            oracle.cosupport(a_f, tau)
            t_cos = time.perf_counter() - t0
        # the log-likelihood needs the co-supports (or analysed vectors) of the
        # listed pixels and of every sample's pixel (work of the front end above)
        need = np.unique(np.concatenate([pix, w.sample_pix])).astype(np.int32)
        a_n = oracle.analyze(w.rgb, w.p, w.mask_sigma, w.omega, pix=need)
        if soft:
            alpha = np.zeros((N, k))
            alpha[need] = a_n
        else:
            masks = np.zeros((N, nw), np.uint64)
            masks[need] = oracle.cosupport(a_n, tau)
        e_f, e_full = n_front * k, N * k
        t_front = (t_an + t_cos) * N / n_front + t_sort * (e_full * math.log2(e_full)) / (e_f * math.log2(e_f))
        how = (f"analysis{'' if soft else ', tau (sort) and masks'} of {n_front} strided pixels "
               f"({t_an + t_sort + t_cos:.2f} s), extrapolated to all {N} pixels ({t_front:.1f} s: analysis and "
               f"masks by pixel count, the sort by n log n)")
    t1 = time.perf_counter()
    if soft:
        oracle.label_loglik_soft(w.rgb, alpha, SIGMA_IOTA, w.sample_pix, w.sample_label, w.L, pix=pix)
    else:
        oracle.label_loglik(w.rgb, masks, k, w.sample_pix, w.sample_label, w.L, pix=pix, joint=joint)
    t_ll = time.perf_counter() - t1
    t_equiv = t_ll + t_front * n_sample / N
    pairs = n_sample * w.M
    return {
        "value": pairs / t_equiv,
        "unit": "pairs/s",
        "cores": oracle.get_threads(),
        "kind": "oracle",
        "sample": (f"FP64 oracle: {how}, scaled to the subset, + Parzen log-likelihood of {n_sample} evenly "
                   f"strided pixels x {w.M} samples ({t_ll:.2f} s)"),
    }


def add_surrogate_args(ap):
    ap.add_argument("--mlp-steps", type=int, default=1000)
    ap.add_argument("--mlp-batch", type=int, default=4096)
    ap.add_argument("--mlp-lr", type=float, default=3e-3)
    ap.add_argument("--fallback-margin", type=float, default=2.0,
                    help="pixels whose two largest surrogate outputs differ by less than this (nats) "
                         "take the exact data term")
    ap.add_argument("--sur-precision", default="bf16", choices=["bf16", "fp32"],
                    help="analysis precision of the surrogate path (its features; the masks of its "
                         "exact targets and fallback are exact either way)")


def surrogate_line(args) -> dict:
    """The learned surrogate at the 2048x2048 workload, per image and measured
    against the plain FP32 exact data term on the same GPU.

    Exact path: co-support step (FP32) and the Parzen log-likelihood of every
    pixel.  Surrogate path: co-support step with the BF16 analysis (the
    analysed vectors are the network's features; the masks are the exact
    ones), exact targets at the 2 % training pixels, training, then inference
    on every pixel with the exact data term for the pixels whose two largest
    outputs differ by less than the fallback margin.  Reported: the pixel
    rate once trained (analysis + inference + fallback), the rate per image
    with targets and training included, the flip rate and |dl| against the
    exact path, and the exact path on a random sample subset sized to the
    surrogate path's whole per-image time (the method without the network at
    equal time)."""
    import numpy as np
    import torch

    from paper_1312_4746_amd import Context, LoglikParams, Mlp, mlp_features
    from paper_1312_4746_amd import surrogate as sg
    from workloads import make_config, mlp_init, mlp_order

    w = make_config(4)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    rgb, om = dev(w.rgb), dev(w.omega)
    spix, slab = dev(w.sample_pix), dev(w.sample_label)
    tpix = dev(w.train_pix)
    prm = LoglikParams(alpha_rho=w.alpha_rho, sigma_c=w.sigma_c, beta_scale=w.beta_scale,
                       rho_floor_px=w.rho_floor_px, colour_levels=w.colour_levels)
    ctx = Context(0)
    nw = (w.k + 63) // 64
    a32 = torch.empty((w.N, w.k), dtype=torch.float32, device="cuda")
    m32 = torch.empty((w.N, nw), dtype=torch.int64, device="cuda")
    asur = torch.empty_like(a32)
    msur = torch.empty_like(m32)
    ll = torch.empty((w.N, w.L), dtype=torch.float32, device="cuda")
    y = torch.empty_like(ll)

    def timed(fn, reps=1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            r = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps, r

    # exact path (the reference)
    front32 = lambda: ctx.cosupport_median(rgb, w.p, w.mask_sigma, om, w.tau_frac, alpha=a32, out=m32)  # noqa: E731
    exact = lambda: ctx.label_loglik(rgb, m32, w.k, spix, slab, w.L, prm, out=ll)  # noqa: E731
    front32()
    exact()
    t_front32, _ = timed(front32, 3)
    t_exact, _ = timed(exact, 1)

    # surrogate path
    steps, batch = args.mlp_steps, args.mlp_batch
    order = dev(mlp_order(len(w.train_pix), steps, batch, seed=w.seed + 101).ravel())
    init = dev(mlp_init(5 + w.k, 128, w.L, seed=w.seed + 100))
    front_s = lambda: ctx.cosupport_median(rgb, w.p, w.mask_sigma, om, w.tau_frac,  # noqa: E731
                                           precision=args.sur_precision, alpha=asur, out=msur)
    front_s()
    t_front_s, _ = timed(front_s, 3)
    ctx.label_loglik(rgb, msur, w.k, spix, slab, w.L, prm, pix_subset=tpix)  # warm-up of the list path
    t_targets, ell = timed(lambda: ctx.label_loglik(rgb, msur, w.k, spix, slab, w.L, prm, pix_subset=tpix))
    t_feat, x = timed(lambda: mlp_features(ctx, rgb, asur, tpix))
    net = Mlp(ctx, 5 + w.k, w.L, init)

    def fit():
        net.fit_output_bias(ell)
        return net.train(x, ell, order, batch, args.mlp_lr)

    t_fit, trace = timed(fit)
    net.infer(rgb, asur, out=y)
    t_infer, _ = timed(lambda: net.infer(rgb, asur, out=y), 5)
    q_plain = sg.compare_to_exact(y, ll)
    net.infer_fallback(rgb, asur, msur, w.k, spix, slab, prm, margin=args.fallback_margin, out=y)
    t_infer_fb, (_, n_exact) = timed(lambda: net.infer_fallback(rgb, asur, msur, w.k, spix, slab, prm,
                                                                margin=args.fallback_margin, out=y), 3)
    q = sg.compare_to_exact(y, ll)
    t_image = t_front_s + t_targets + t_feat + t_fit + t_infer_fb

    # the method without the network at equal time: the exact path on a random
    # sample subset sized so that front + Parzen take the surrogate path's time
    frac_eq = max(0.0, min(1.0, (t_image - t_front32) / t_exact))
    m_eq = max(w.L, int(w.M * frac_eq))
    gen = torch.Generator().manual_seed(w.seed + 102)
    sp2, sl2 = sg.equal_time_subset(spix, slab, w.L, m_eq, gen)
    ll2 = torch.empty_like(ll)
    ctx.label_loglik(rgb, m32, w.k, sp2, sl2, w.L, prm, out=ll2)
    t_sub, _ = timed(lambda: ctx.label_loglik(rgb, m32, w.k, sp2, sl2, w.L, prm, out=ll2), 1)
    q_sub = sg.compare_to_exact(ll2, ll)
    tr = trace.cpu().numpy()
    t_exact_total = t_front32 + t_exact
    out = {
        "metric": "surrogate px/s at <=0.5% label-argmax flips",
        "value": w.N / (t_front_s + t_infer_fb),
        "unit": "px/s",
        "n_gpus": 1,
        "steps": 3,
        "warmup": 1,
        "ms_per_step": (t_front_s + t_infer_fb) * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": f"{args.sur_precision}+f32",
        "data": "synthetic",
        "config": {"workload": w.name, "H": w.H, "W": w.W, "k": w.k, "labels": w.L, "samples": w.M,
                   "pixels": w.N, "train_pixels": int(len(w.train_pix)), "parallelism": "1 GPU"},
        "surrogate": {
            "flip_rate": q["flip_rate"],
            "meets_0p5pct": q["flip_rate"] <= 0.005,
            "mean_abs_dl": q["mean_abs_dl"],
            "mean_abs_dl_within_20_nats": q["mean_abs_dl_within_20_nats"],
            "fallback": {"margin_nats": args.fallback_margin, "pixels": n_exact,
                         "fraction": n_exact / w.N},
            "without_fallback": {"flip_rate": q_plain["flip_rate"],
                                 "mean_abs_dl_within_20_nats": q_plain["mean_abs_dl_within_20_nats"]},
            "analysis_precision": args.sur_precision,
            "ms": {"front": t_front_s * 1e3, "targets": t_targets * 1e3, "features": t_feat * 1e3,
                   "fit": t_fit * 1e3, "infer": t_infer * 1e3, "infer_with_fallback": t_infer_fb * 1e3,
                   "per_image": t_image * 1e3},
            "px_per_s_trained": w.N / (t_front_s + t_infer_fb),
            "px_per_s_per_image_incl_fit": w.N / t_image,
            "train": {"steps": steps, "batch": batch, "lr": args.mlp_lr,
                      "loss_first": float(tr[:20].mean()), "loss_last": float(tr[-20:].mean())},
        },
        "exact": {"px_per_s": w.N / t_exact_total, "front_ms": t_front32 * 1e3, "loglik_ms": t_exact * 1e3,
                  "pairs_per_s": w.N * w.M / t_exact},
        "speedup_per_image_incl_fit": t_exact_total / t_image,
        "speedup_trained": t_exact_total / (t_front_s + t_infer_fb),
        "equal_time_exact": {"samples": int(sp2.numel()), "sample_fraction": sp2.numel() / w.M,
                             "ms": (t_front32 + t_sub) * 1e3, "flip_rate": q_sub["flip_rate"],
                             "mean_abs_dl_within_20_nats": q_sub["mean_abs_dl_within_20_nats"]},
    }
    net.close()
    ctx.close()
    return out


def mean_dice(labels, truth, L: int) -> float:
    """Mean over the labels of the Dice score 2 |A n B| / (|A| + |B|) (evaluation)."""
    import numpy as np
    d = []
    for i in range(L):
        a, b = labels == i, truth == i
        den = int(a.sum() + b.sum())
        d.append(2.0 * int((a & b).sum()) / den if den else 1.0)
    return float(np.mean(d))


def segment_line(args, config: int = 1) -> dict:
    """Segmentation by convex relaxation (Sec. 4) on the exact data term of
    workload `config`: the primal-dual iteration's time per iteration against
    the HBM roofline (algorithmic bytes per pixel and label: read u_bar, xi_x,
    xi_y, u, f; write xi_x, xi_y, u, u_bar: 36 B in FP32), the energies and the
    relaxation gap, Dice against the synthetic regions, and the FP64 oracle's
    iteration on the host."""
    import numpy as np
    import torch

    from paper_1312_4746_amd import Context, LoglikParams, SegmentParams
    from workloads import make_config

    w = make_config(config)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    rgb = dev(w.rgb)
    prm = LoglikParams(alpha_rho=w.alpha_rho, sigma_c=w.sigma_c, beta_scale=w.beta_scale,
                       rho_floor_px=w.rho_floor_px, colour_levels=w.colour_levels)
    ctx = Context(0)
    _, masks, _ = ctx.cosupport_median(rgb, w.p, w.mask_sigma, dev(w.omega), w.tau_frac)
    ll = ctx.label_loglik(rgb, masks, w.k, dev(w.sample_pix), dev(w.sample_label), w.L, prm)
    sp = SegmentParams(lam=args.seg_lambda, nu=0.0, iterations=args.seg_iters, precision="fp32")
    ctx.segment(rgb, ll, sp)  # warm-up
    torch.cuda.synchronize()
    ctx.profile_only("pd_iter")
    ctx.profile_sample(4)
    ctx.profile_enable(True)
    t0 = time.perf_counter()
    lab, _, st = ctx.segment(rgb, ll, sp)
    torch.cuda.synchronize()
    t_solve = time.perf_counter() - t0
    it_ms, it_n = ctx.profile_read("pd_iter")
    ctx.profile_enable(False)
    ctx.profile_sample(1)
    ctx.profile_only(None)
    avg_it = it_ms / 1e3 / max(it_n, 1)
    bytes_it = w.N * w.L * 36 + w.N * 4
    lab_np = lab.cpu().numpy().reshape(w.H, w.W)
    ll_np = ll.cpu().numpy()
    dice0 = mean_dice(np.argmax(ll_np, 1).reshape(w.H, w.W), w.region, w.L)
    dice1 = mean_dice(lab_np, w.region, w.L)
    ctx.close()
    cpu = None
    if not args.no_cpu:
        # the oracle's iteration (numpy FP64) on the same data term, a few iterations timed
        from oracle import segment as osg
        f = osg.data_term(ll_np.astype(np.float64), w.H, w.W)
        g, _ = osg.edge_weight(w.rgb)
        n_cpu = 10
        t0 = time.perf_counter()
        osg.solve(f, g, lam=args.seg_lambda, iterations=n_cpu)
        t_cpu = (time.perf_counter() - t0) / n_cpu
        cpu = {"value": 1.0 / t_cpu, "unit": "iterations/s", "cores": 1, "kind": "oracle",
               "sample": f"FP64 numpy oracle, {n_cpu} iterations on {w.H}x{w.W}x{w.L} ({t_cpu * 1e3:.1f} ms each)"}
    return {
        "metric": "primal-dual iterations/s",
        "value": 1.0 / avg_it,
        "unit": "iterations/s",
        "workload": w.name, "H": w.H, "W": w.W, "labels": w.L,
        "iterations": args.seg_iters, "lambda": args.seg_lambda, "dtype": "f32",
        "ms_per_iteration": avg_it * 1e3, "solve_ms": t_solve * 1e3,
        "roofline": {"bound": "hbm", "achieved": bytes_it / avg_it / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                     "frac": bytes_it / avg_it / PEAK_HBM, "traffic": None, "kernel": "k_pd_iter",
                     "bytes_per_iteration": bytes_it},
        "energies": st,
        "relaxation_gap": (st["binary"] - st["dual"]) / abs(st["dual"]),
        "dice_vs_regions": {"pointwise_argmax": dice0, "segmentation": dice1},
        "cpu_baseline": cpu,
    }


def partition_scores(labels, truth) -> dict:
    """Rand index and variation of information (bits) between two labellings
    (evaluation of a segmentation against the synthetic regions)."""
    import numpy as np
    a = np.asarray(labels).ravel().astype(np.int64)
    b = np.asarray(truth).ravel().astype(np.int64)
    n = a.size
    ka, kb = int(a.max()) + 1, int(b.max()) + 1
    cont = np.bincount(a * kb + b, minlength=ka * kb).reshape(ka, kb).astype(np.float64)
    ra, rb = cont.sum(1), cont.sum(0)
    c2 = lambda v: (v * (v - 1) / 2.0).sum()  # noqa: E731
    disagree = c2(ra) + c2(rb) - 2.0 * c2(cont)
    ri = 1.0 - disagree / (n * (n - 1) / 2.0)
    p = cont / n
    nz = p > 0
    h = lambda q: -(q[q > 0] * np.log2(q[q > 0])).sum()  # noqa: E731
    voi = 2.0 * (-(p[nz] * np.log2(p[nz])).sum()) - h(ra / n) - h(rb / n)
    return {"rand_index": float(ri), "voi_bits": float(voi), "segments": int((ra > 0).sum())}


def unsup_line(args, config: int = 1) -> dict:
    """Unsupervised segmentation (Sec. 3.1, Sec. 3.2 eq:mdl, Sec. 4) on
    workload `config`: co-supports, k-means on colours and k-medians on
    co-supports into 4 x 4 product classes (the paper's 16 initial regions),
    their likelihoods, then the convex relaxation with the label cost
    (lambda = 6, nu = 1100 as in the paper's BSDS runs); time per image, the
    labels kept, and the Rand index / variation of information against the
    synthetic regions."""
    import numpy as np
    import torch

    from paper_1312_4746_amd import Context, SegmentParams, UnsupParams
    from workloads import make_config, unsup_init

    w = make_config(config)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    rgb, om = dev(w.rgb), dev(w.omega)
    ctx = Context(0)
    ic, it = unsup_init(w.N, 4, 4, w.seed + 200)
    up = UnsupParams(colour_classes=4, texture_classes=4, iterations=10, sigma_c=w.sigma_c, beta=2.0)
    sp = SegmentParams(lam=6.0, nu=1100.0, iterations=args.seg_iters, precision="fp32")

    def run():
        _, m, _ = ctx.cosupport_median(rgb, w.p, w.mask_sigma, om, w.tau_frac)
        ll, _ = ctx.unsupervised_loglik(rgb, m, w.k, ic, it, up)
        return ctx.segment(rgb, ll, sp)

    run()
    torch.cuda.synchronize()
    reps = 3
    t0 = time.perf_counter()
    for _ in range(reps):
        lab, _, st = run()
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / reps
    sc = partition_scores(lab.cpu().numpy(), w.region)
    ctx.close()
    return {"metric": "unsupervised segmentations/s", "value": 1.0 / t, "unit": "images/s", "workload": w.name,
            "ms_per_image": t * 1e3, "classes": 16, "lambda": 6.0, "nu": 1100.0, "iterations": args.seg_iters,
            "labels_used": st["labels_used"], "relaxation_gap": (st["binary"] - st["dual"]) / abs(st["dual"]),
            "vs_regions": sc}


def counter_profile(kernel: str, workload: str, digest_of=None):
    """The committed counter summary of `kernel` at `workload`
    (profiles/<kernel>_<workload>_counters.json), or None when it is absent or
    was taken on another source of the kernel."""
    prof = load_profile(f"{kernel}_{workload}_counters.json")
    if not prof or prof.get("workload") != workload:
        return None
    if digest_of is not None and prof.get("source_digest") != digest_of():
        return None
    return prof


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--config", type=int, default=3,
                    help="workload: 3 large (default), 5 large with BF16 analysis, 1 BSDS-sized, "
                         "2 BSDS-sized with BF16 analysis, 0 tiny, 4 the surrogate case alone")
    ap.add_argument("--cpu-sample", type=int, default=0,
                    help="pixels of the oracle's log-likelihood sample (0: 2048 for images above "
                         "131072 pixels, else 32768)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true",
                    help="leave out the surrogate leg (2048x2048) of the headline line")
    ap.add_argument("--no-segment", action="store_true",
                    help="leave out the segmentation leg (primal-dual iteration) of the headline line")
    ap.add_argument("--segment", action="store_true",
                    help="only the segmentation leg (primal-dual iteration) on --config's data term")
    ap.add_argument("--seg-iters", type=int, default=300)
    ap.add_argument("--unsup", action="store_true",
                    help="only the unsupervised segmentation leg on --config's image")
    ap.add_argument("--seg-lambda", type=float, default=1.0)
    ap.add_argument("--float-colours", action="store_true",
                    help="pass the colours as plain floats (colour_levels 0: the colour term on the VALU) "
                         "instead of the workload's 8-bit levels")
    ap.add_argument("--soft", action="store_true",
                    help="the joint form with smooth co-supports (sigma 0.01) of the stored "
                         "analysed vectors")
    ap.add_argument("--joint", action="store_true",
                    help="the paper's combination: colour/location Parzen density times the "
                         "texture posterior against label representatives")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (5 times), to scale the HBM "
                         "byte counters of a profiler run")
    add_surrogate_args(ap)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the data term runs on a single MI355X "
              "(multi-GPU sharding is a design note, not built); run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    if args.copy_calibration:
        import torch
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_per_launch_read": n * 4, "written": n * 4, "launches": 5}))
        return
    if args.config == 4:
        print(json.dumps(surrogate_line(args)))
        return
    if args.segment:
        print(json.dumps(segment_line(args, args.config)))
        return
    if args.unsup:
        print(json.dumps(unsup_line(args, args.config)))
        return

    import numpy as np
    import torch

    from paper_1312_4746_amd import Context, LoglikParams
    from workloads import make_config

    w = make_config(args.config)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    rgb, om = dev(w.rgb), dev(w.omega)
    spix, slab = dev(w.sample_pix), dev(w.sample_label)
    levels = 0 if args.float_colours else w.colour_levels
    prm = LoglikParams(alpha_rho=w.alpha_rho, sigma_c=w.sigma_c, beta_scale=w.beta_scale,
                       rho_floor_px=w.rho_floor_px, colour_levels=levels)
    ctx = Context(0)
    alpha = torch.empty((w.N, w.k), dtype=torch.float32, device="cuda")
    masks = torch.empty((w.N, (w.k + 63) // 64), dtype=torch.int64, device="cuda")
    ll = torch.empty((w.N, w.L), dtype=torch.float32, device="cuda")

    tau = torch.empty(1, dtype=torch.float64, device="cuda")

    def step():
        # analysis, exact tau = frac * median|a| and the masks (no host round
        # trip), then the per-label log-likelihoods of every pixel
        ctx.cosupport_median(rgb, w.p, w.mask_sigma, om, w.tau_frac, precision=w.precision, alpha=alpha,
                             out=masks, tau=tau)
        ctx.label_loglik(rgb, masks, w.k, spix, slab, w.L, prm, out=ll, joint=args.joint)

    def step_soft():
        # analysis with the analysed vectors stored, then the joint form on
        # their smooth co-supports (no threshold, no masks)
        ctx.analyze_patches(rgb, w.p, w.mask_sigma, om, precision=w.precision, out=alpha)
        ctx.label_loglik_soft(rgb, alpha, SIGMA_IOTA, spix, slab, w.L, prm, out=ll)

    if args.soft:
        step = step_soft  # noqa: F811

    print(f"[bench] {w.name}: {args.warmup} warm-up + {args.steps} timed steps", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # inside the timed region only the Parzen kernel carries events, on one
    # launch in PARZEN_EVENT_PERIOD (each recorded event adds a short bubble
    # to the stream)
    ctx.profile_only("parzen")
    ctx.profile_sample(PARZEN_EVENT_PERIOD)
    ctx.profile_enable(True)
    torch.cuda.synchronize()
    # steps run back to back (no host synchronisation between them)
    t0 = time.perf_counter()
    for i in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    lse_stats = ctx.last_loglik_stats()
    parzen_ms, parzen_n = ctx.profile_read("parzen")
    ctx.profile_sample(1)
    # the per-step spread, from events between steps outside the timed region
    spread_steps = min(args.steps, 20)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(spread_steps + 1)]
    ev[0].record()
    for i in range(spread_steps):
        step()
        ev[i + 1].record()
    torch.cuda.synchronize()
    per_step = [ev[i].elapsed_time(ev[i + 1]) / 1e3 for i in range(spread_steps)]
    # every stage's kernel time, from a few more steps outside the timed region
    stage_steps = 3
    ctx.profile_only(None)
    ctx.profile_enable(True)
    for _ in range(stage_steps):
        step()
    stage_names = ["analyze", "tau_select", "cosupport", "tau_exact", "cosupport_fix", "thresholds", "samples",
                   "edt", "stream", "texture_rep", "coef", "parzen", "parzen_fixup", "texture", "normalise"]
    stages = {}
    for nm in stage_names:
        ms_, n_ = ctx.profile_read(nm)
        if n_:
            stages[nm] = ms_ / stage_steps
    analyze_ms, analyze_n = ctx.profile_read("analyze")
    ctx.profile_enable(False)

    ms_per_step = dt * 1e3 / args.steps
    pairs = w.N * w.M
    value = pairs / (ms_per_step / 1e3)

    avg_parzen_s = parzen_ms / 1e3 / max(parzen_n, 1)
    tex_in_sum = not (args.joint or args.soft)
    ops_pp = parzen_ops_per_pair(w.k, tex_in_sum)
    achieved = pairs * ops_pp / avg_parzen_s
    # the kernel that ran: the 32 x 32 form with colour levels, the 16 x 16 one with float colours
    parzen_kernel = "k_parzen_mfma32" if levels else "k_parzen_mfma"
    prof = counter_profile(parzen_kernel, w.name, kernel_source_digest) if tex_in_sum else None
    traffic = prof.get("bytes_per_launch") if prof else None
    counters = None
    if prof:
        counters = {k_: prof.get(k_) for k_ in ("valu_issue_frac", "valu_busy_frac", "mfma_busy_frac",
                                                "valu_insts_per_pair", "avg_duration_us")}
        if traffic:
            counters["hbm_gbs_live"] = traffic / avg_parzen_s / 1e9
            counters["hbm_frac"] = traffic / avg_parzen_s / PEAK_HBM
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32_VECTOR / 1e12,
                "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_VECTOR, "traffic": traffic,
                "kernel": parzen_kernel, "avg_launch_ms": avg_parzen_s * 1e3, "ops_per_pair": ops_pp,
                "ops_model": "direct evaluation per pair: location 4, colour 6, XOR+popcount 2 ceil(k/32), "
                             "convert+exponent 4, log-sum-exp 3, v_exp_f32 as 4 slots",
                "note": "algorithmic rate against the FP32 vector peak; the kernel forms the texture, location "
                        "(and with colour levels the colour) terms as exact products on the matrix cores, so "
                        "the rate can pass the vector peak: unit utilisations are under counters",
                "counters": counters}
    avg_an = analyze_ms / 1e3 / max(analyze_n, 1)
    gemm_flops = 2.0 * w.k * w.n * w.N
    an_prof = counter_profile("k_analyze", w.name)
    extra = {
        "analyze_mfma": {"avg_launch_ms": avg_an * 1e3, "achieved_tflops": gemm_flops / avg_an / 1e12,
                         "peak_tflops": PEAK_MFMA[w.precision] / 1e12,
                         "frac": gemm_flops / avg_an / PEAK_MFMA[w.precision],
                         "mfma_busy_frac": an_prof.get("mfma_busy_frac") if an_prof else None},
        "stage_ms_per_step": stages,
        "px_per_s": w.N / (ms_per_step / 1e3),
        "step_ms_min_median_max": [min(per_step) * 1e3, float(np.median(per_step)) * 1e3,
                                   max(per_step) * 1e3],
        "lse_reference_events": lse_stats,
    }
    if w.precision == "bf16":
        extra["precision_sweep"] = precision_sweep(ctx, w, rgb, om, alpha, spix, slab, prm)
    ctx.close()
    del alpha, masks, ll

    cpu = None
    if not args.no_cpu:
        print("[bench] oracle baseline on the host", file=sys.stderr, flush=True)
        n_cpu = args.cpu_sample or (2048 if w.N > 131072 else 32768)
        cpu = cpu_baseline(w, min(n_cpu, w.N), joint=args.joint, soft=args.soft)

    sur = None
    if not args.no_surrogate and not (args.joint or args.soft):
        print("[bench] surrogate leg (2048x2048)", file=sys.stderr, flush=True)
        full = surrogate_line(args)
        sur = {k_: full[k_] for k_ in ("value", "unit", "ms_per_step")}
        sur.update({"workload": full["config"]["workload"], **full["surrogate"]})
        for k_ in ("exact", "speedup_per_image_incl_fit", "speedup_trained", "equal_time_exact"):
            sur[k_] = full[k_]

    seg = None
    if not args.no_segment and not (args.joint or args.soft):
        print("[bench] segmentation leg (BSDS-sized data term)", file=sys.stderr, flush=True)
        seg = segment_line(args, 1)
        print("[bench] unsupervised leg (BSDS-sized image)", file=sys.stderr, flush=True)
        seg["unsupervised"] = unsup_line(args, 1)

    out = {
        "metric": "data-term pixel x sample pairs/s",
        "value": value,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if w.precision == "fp32" else "bf16+f32",
        "data": "synthetic",
        "config": {"workload": w.name + ("+soft" if args.soft else "+joint" if args.joint else ""),
                   "H": w.H, "W": w.W, "p": w.p, "k": w.k, "labels": w.L,
                   "texture": ("smooth co-supports, median representatives (eq:map_tsm, eq:joined)"
                               if args.soft else "label representatives (eq:joined)" if args.joint
                               else "per sample in the sum"),
                   "colours": (f"{levels + 1} levels per channel (colour term on the matrix cores)" if levels
                               else "floats (colour term on the VALU)"),
                   "samples": w.M, "pixels": w.N, "pairs": pairs, "parallelism": "1 GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "surrogate": sur,
        "segmentation": seg,
        "extra": extra,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
