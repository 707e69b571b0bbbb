"""Per-image learned surrogate of the data term: train on exact
log-likelihoods at sampled pixels, infer on every pixel, compare against the
exact path.

Every computation of the method runs in the library (exact targets by
cs_label_loglik on the training pixels, input rows by cs_mlp_features,
training and inference by the surrogate kernels); torch only holds device
memory and compares outputs (argmax flips, absolute differences).
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import torch

from .binding import Context, LoglikParams, Mlp, mlp_features

CLIP_NATS = 20.0


@dataclasses.dataclass
class SurrogateFit:
    net: Mlp
    loss_trace: torch.Tensor
    steps: int


def fit(ctx: Context, rgb: torch.Tensor, alpha: torch.Tensor, masks: torch.Tensor, k: int,
        sample_pix: torch.Tensor, sample_label: torch.Tensor, L: int, params: LoglikParams,
        train_pix: torch.Tensor, init_params: torch.Tensor, order: torch.Tensor, batch: int,
        lr: float = 1e-3) -> SurrogateFit:
    """Exact targets at train_pix (int32), then Adam over the batches of
    `order` (int32 row indices into the training rows, a multiple of batch)."""
    ell = ctx.label_loglik(rgb, masks, k, sample_pix, sample_label, L, params, pix_subset=train_pix)
    x = mlp_features(ctx, rgb, alpha, train_pix)
    net = Mlp(ctx, 5 + k, L, init_params)
    net.fit_output_bias(ell)
    trace = net.train(x, ell, order, batch, lr)
    return SurrogateFit(net=net, loss_trace=trace, steps=int(order.numel() // batch))


def compare_to_exact(ell_sur: torch.Tensor, ell_exact: torch.Tensor) -> dict:
    """Label-argmax flip rate (ties to the lowest label on both sides), mean
    |delta l| over all labels, and over the labels within CLIP_NATS of the
    pixel's exact maximum (the range the surrogate is trained to match)."""
    a = torch.argmax(ell_sur, dim=1)
    b = torch.argmax(ell_exact, dim=1)
    d = (ell_sur - ell_exact).abs()
    near = ell_exact >= ell_exact.max(dim=1, keepdim=True).values - CLIP_NATS
    return {
        "flip_rate": float((a != b).float().mean()),
        "mean_abs_dl": float(d.mean()),
        "mean_abs_dl_within_20_nats": float(d[near].mean()),
        "pixels": int(ell_exact.shape[0]),
    }


def equal_time_subset(sample_pix: torch.Tensor, sample_label: torch.Tensor, L: int, m: int,
                      generator: Optional[torch.Generator] = None):
    """A random subset of about m scribble samples that keeps at least one
    sample of every label (per-label shares proportional to the label's
    count), for the exact path at reduced cost."""
    keep = []
    counts = torch.bincount(sample_label.long(), minlength=L).cpu()
    total = int(counts.sum())
    for lab in range(L):
        idx = torch.nonzero(sample_label == lab).flatten()
        want = max(1, int(round(m * int(counts[lab]) / total)))
        want = min(want, idx.numel())
        perm = torch.randperm(idx.numel(), generator=generator, device="cpu")[:want].to(idx.device)
        keep.append(idx[perm])
    sel = torch.cat(keep)
    return sample_pix[sel].contiguous(), sample_label[sel].contiguous()
