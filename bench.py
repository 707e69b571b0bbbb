"""Benchmark of the co-sparse data term on one MI355X.

One step = the whole data-term path over one synthetic image: analysed
vectors (MFMA), exact threshold tau, co-support masks, and the per-pixel,
per-label log-likelihood (distance transform + Parzen sum).  The workload is
the BSDS-sized case: 481x321 RGB, 7x7 patches, k = 98, 10 labels, 7,720
scribble samples, FP32.  Inputs are resident in HBM before timing starts.

Prints one JSON line with the whole-job throughput (pixel x sample pairs/s),
the roofline of the dominant kernel (the Parzen sum, measured with HIP events
on the stream it runs on) and the FP64 oracle timed on the host on a bounded
sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X: 256 CUs at 2.4 GHz; the published FP32 vector rate 157.3 TFLOP/s is
# 128 FMA lanes per clock per CU, i.e. 7.86e13 single-rate VALU lane-operations
# per second; HBM3E 8 TB/s; FP32 matrix 157.3 TFLOP/s; BF16 dense 2.5 PFLOP/s.
PEAK_LANE_OPS = 157.3e12 / 2
PEAK_HBM = 8.0e12
# the Parzen kernel carries timing events on one launch in this many inside the timed region
# smooth co-support map exp(-a^2 / sigma) of the paper's experiments
SIGMA_IOTA = 0.01
PARZEN_EVENT_PERIOD = 8
PEAK_MFMA = {"fp32": 157.3e12, "bf16": 2.5e15}


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


def load_traffic(name: str):
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            return json.load(f)
    except Exception:
        return None


def kernel_source_digest() -> str:
    """Digest of the Parzen kernel's source and of its argument struct (the
    traffic counters stay valid while neither changes)."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_1312_4746_amd", "csrc")
    h = hashlib.sha256()
    with open(os.path.join(csrc, "k_parzen_mfma.hip"), "rb") as fh:
        h.update(fh.read())
    with open(os.path.join(csrc, "cs_internal.h")) as fh:
        hdr = fh.read()
    a = hdr.index("struct ParzenFastArgs")
    h.update(hdr[a:hdr.index("};", a)].encode())
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


def cpu_baseline(w, n_sample: int, joint: bool = False, soft: bool = False):
    """The FP64 oracle on the host: full-image analysis, tau and masks (needed
    for any pixel), then the Parzen log-likelihood on a strided subset of
    pixels; the per-pixel front-end time is scaled to the subset."""
    import numpy as np

    import oracle
    oracle.lib()
    t0 = time.perf_counter()
    alpha = oracle.analyze(w.rgb, w.p, w.mask_sigma, w.omega)
    if not soft:  # the smooth form needs no threshold and no masks
        tau, _ = oracle.tau_median(alpha, w.tau_frac)
        masks = oracle.cosupport(alpha, tau)
    t_front = time.perf_counter() - t0
    pix = np.linspace(0, w.N - 1, n_sample).astype(np.int32)
    t1 = time.perf_counter()
    if soft:
        oracle.label_loglik_soft(w.rgb, alpha, SIGMA_IOTA, w.sample_pix, w.sample_label, w.L, pix=pix)
    else:
        oracle.label_loglik(w.rgb, masks, w.k, w.sample_pix, w.sample_label, w.L, pix=pix, joint=joint)
    t_ll = time.perf_counter() - t1
    t_equiv = t_ll + t_front * n_sample / w.N
    pairs = n_sample * w.M
    return {
        "value": pairs / t_equiv,
        "unit": "pairs/s",
        "cores": oracle.get_threads(),
        "kind": "oracle",
        "sample": (f"FP64 oracle: analysis{'' if soft else ', tau and masks'} of all {w.N} pixels ({t_front:.2f} s, "
                   f"scaled to the subset) + Parzen log-likelihood of {n_sample} evenly strided "
                   f"pixels x {w.M} samples ({t_ll:.2f} s)"),
    }


def surrogate_bench(args):
    """Learned surrogate at the 2048x2048 workload: exact data term on every
    pixel (the reference), exact targets at the 2 % training pixels, training,
    inference on every pixel, flip rate and the equal-time comparison."""
    import numpy as np
    import torch

    from paper_1312_4746_amd import Context, LoglikParams
    from paper_1312_4746_amd import surrogate as sg
    from workloads import make_config, mlp_init, mlp_order

    w = make_config(args.config)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    rgb, om = dev(w.rgb), dev(w.omega)
    spix, slab = dev(w.sample_pix), dev(w.sample_label)
    tpix = dev(w.train_pix)
    prm = LoglikParams(alpha_rho=w.alpha_rho, sigma_c=w.sigma_c, beta_scale=w.beta_scale,
                       rho_floor_px=w.rho_floor_px)
    ctx = Context(0)
    alpha = torch.empty((w.N, w.k), dtype=torch.float32, device="cuda")
    masks = torch.empty((w.N, (w.k + 63) // 64), dtype=torch.int64, device="cuda")
    ll = torch.empty((w.N, w.L), dtype=torch.float32, device="cuda")

    def timed(fn, reps=1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            r = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps, r

    def front():
        ctx.analyze_patches(rgb, w.p, w.mask_sigma, om, precision=w.precision, out=alpha)
        tau = ctx.tau_median(rgb, w.p, w.mask_sigma, om, alpha, w.tau_frac, precision=w.precision)
        ctx.cosupport(rgb, w.p, w.mask_sigma, om, tau, precision=w.precision, out=masks, alpha=alpha)

    front()  # warm-up
    t_front, _ = timed(front, 2)
    t_analyze, _ = timed(lambda: ctx.analyze_patches(rgb, w.p, w.mask_sigma, om, precision=w.precision,
                                                     out=alpha), 2)
    front()
    exact = lambda: ctx.label_loglik(rgb, masks, w.k, spix, slab, w.L, prm, out=ll)  # noqa: E731
    exact()
    t_exact, _ = timed(exact, 1)

    batch, steps = args.mlp_batch, args.mlp_steps
    order = dev(mlp_order(len(w.train_pix), steps, batch, seed=w.seed + 101).ravel())
    init = dev(mlp_init(5 + w.k, 128, w.L, seed=w.seed + 100))
    t_fit, fit = timed(lambda: sg.fit(ctx, rgb, alpha, masks, w.k, spix, slab, w.L, prm, tpix, init, order,
                                      batch, args.mlp_lr))
    net = fit.net
    y = torch.empty((w.N, w.L), dtype=torch.float32, device="cuda")
    net.infer(rgb, alpha, out=y)
    reps = 5
    t_infer, _ = timed(lambda: net.infer(rgb, alpha, out=y), reps)
    quality = sg.compare_to_exact(y, ll)

    # equal-time exact path: a sample subset sized to the surrogate's time
    m_eq = max(w.L, int(w.M * t_infer / t_exact))
    gen = torch.Generator().manual_seed(w.seed + 102)
    sp2, sl2 = sg.equal_time_subset(spix, slab, w.L, m_eq, gen)
    ll2 = torch.empty_like(ll)
    ctx.label_loglik(rgb, masks, w.k, sp2, sl2, w.L, prm, out=ll2)
    t_sub, _ = timed(lambda: ctx.label_loglik(rgb, masks, w.k, sp2, sl2, w.L, prm, out=ll2), 1)
    q_sub = sg.compare_to_exact(ll2, ll)
    trace = fit.loss_trace.cpu().numpy()

    out = {
        "metric": "surrogate px/s at <=0.5% label-argmax flips",
        "value": w.N / t_infer,
        "unit": "px/s",
        "n_gpus": 1,
        "steps": reps,
        "warmup": 1,
        "ms_per_step": t_infer * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16+f32",
        "data": "synthetic",
        "config": {"workload": w.name, "H": w.H, "W": w.W, "k": w.k, "labels": w.L, "samples": w.M,
                   "pixels": w.N, "train_pixels": int(len(w.train_pix)), "parallelism": "1 GPU"},
        "surrogate": {
            "flip_rate": quality["flip_rate"],
            "meets_0p5pct": quality["flip_rate"] <= 0.005,
            "mean_abs_dl": quality["mean_abs_dl"],
            "mean_abs_dl_within_20_nats": quality["mean_abs_dl_within_20_nats"],
            "infer_ms": t_infer * 1e3,
            "train": {"steps": steps, "batch": batch, "lr": args.mlp_lr,
                      "fit_ms_incl_targets": t_fit * 1e3,
                      "loss_first": float(trace[:20].mean()), "loss_last": float(trace[-20:].mean())},
        },
        "exact": {"px_per_s": w.N / (t_front + t_exact), "front_ms": t_front * 1e3,
                  "loglik_ms": t_exact * 1e3, "pairs_per_s": w.N * w.M / t_exact},
        "speedup_vs_exact_data_term": (t_front + t_exact) / (t_analyze + t_infer),
        "equal_time_exact": {"samples": int(sp2.numel()), "ms": t_sub * 1e3, "flip_rate": q_sub["flip_rate"],
                             "mean_abs_dl_within_20_nats": q_sub["mean_abs_dl_within_20_nats"]},
    }
    print(json.dumps(out))
    net.close()
    ctx.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--config", type=int, default=1)
    ap.add_argument("--cpu-sample", type=int, default=32768)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--soft", action="store_true",
                    help="the joint form with smooth co-supports (sigma 0.01) of the stored "
                         "analysed vectors")
    ap.add_argument("--joint", action="store_true",
                    help="the paper's combination: colour/location Parzen density times the "
                         "texture posterior against label representatives")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (5 times), to scale the HBM "
                         "byte counters of a profiler run")
    ap.add_argument("--mlp-steps", type=int, default=3000)
    ap.add_argument("--mlp-batch", type=int, default=4096)
    ap.add_argument("--mlp-lr", type=float, default=1e-3)
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
        surrogate_bench(args)
        return

    import numpy as np
    import torch

    from paper_1312_4746_amd import Context, LoglikParams
    from workloads import make_config

    w = make_config(args.config)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    rgb, om = dev(w.rgb), dev(w.omega)
    spix, slab = dev(w.sample_pix), dev(w.sample_label)
    prm = LoglikParams(alpha_rho=w.alpha_rho, sigma_c=w.sigma_c, beta_scale=w.beta_scale,
                       rho_floor_px=w.rho_floor_px)
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
    spread_steps = min(args.steps, 50)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(spread_steps + 1)]
    ev[0].record()
    for i in range(spread_steps):
        step()
        ev[i + 1].record()
    torch.cuda.synchronize()
    per_step = [ev[i].elapsed_time(ev[i + 1]) / 1e3 for i in range(spread_steps)]
    # the other stages' kernel times, from a few more steps outside the timed region
    stage_steps = 3
    ctx.profile_only(None)
    ctx.profile_enable(True)
    for _ in range(stage_steps):
        step()
    analyze_ms, analyze_n = ctx.profile_read("analyze")
    cos_ms, cos_n = ctx.profile_read("cosupport")
    edt_ms, _ = ctx.profile_read("edt")
    ctx.profile_enable(False)

    ms_per_step = dt * 1e3 / args.steps
    pairs = w.N * w.M
    value = pairs / (ms_per_step / 1e3)

    avg_parzen_s = parzen_ms / 1e3 / max(parzen_n, 1)
    tex_in_sum = not (args.joint or args.soft)
    ops = pairs * parzen_ops_per_pair(w.k, tex_in_sum)
    achieved = ops / avg_parzen_s
    traffic = None
    tr = load_traffic("parzen_bsds_traffic.json")
    # counters taken on this kernel source and this workload only
    if (tr and not (args.joint or args.soft) and tr.get("source_digest") == kernel_source_digest()
            and tr.get("workload") == w.name):
        traffic = tr.get("bytes_per_launch")
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_LANE_OPS / 1e12,
                "unit": "TOP/s", "frac": achieved / PEAK_LANE_OPS, "traffic": traffic,
                "kernel": "k_parzen_mfma", "avg_launch_ms": avg_parzen_s * 1e3,
                "ops_per_pair": parzen_ops_per_pair(w.k, tex_in_sum)}
    avg_an = analyze_ms / 1e3 / max(analyze_n, 1)
    gemm_flops = 2.0 * w.k * w.n * w.N
    extra = {
        "analyze_mfma": {"avg_launch_ms": avg_an * 1e3, "achieved_tflops": gemm_flops / avg_an / 1e12,
                         "peak_tflops": PEAK_MFMA[w.precision] / 1e12,
                         "frac": gemm_flops / avg_an / PEAK_MFMA[w.precision]},
        "cosupport_avg_launch_ms": cos_ms / max(cos_n, 1),
        "edt_ms_per_step": edt_ms / stage_steps,
        "px_per_s": w.N / (ms_per_step / 1e3),
        "step_ms_min_median_max": [min(per_step) * 1e3, float(np.median(per_step)) * 1e3,
                                   max(per_step) * 1e3],
        "lse_reference_events": lse_stats,
    }
    if w.precision == "bf16":
        extra["precision_sweep"] = precision_sweep(ctx, w, rgb, om, alpha, spix, slab, prm)

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(w, min(args.cpu_sample, w.N), joint=args.joint, soft=args.soft)

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
                   "samples": w.M, "pixels": w.N, "pairs": pairs, "parallelism": "1 GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(out))
    ctx.close()


if __name__ == "__main__":
    main()
