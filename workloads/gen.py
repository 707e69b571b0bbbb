"""Seeded generator of synthetic textured images, analysis operators and
scribble samples.

The paper evaluates on the Graz interactive benchmark and on BSDS300
(Sec. 5); neither is available here, so these images stand in for them:
Voronoi regions, each with its own mean colour and an oriented sinusoid
texture (plus band-limited noise for the large case), plus i.i.d. Gaussian
noise; the configured workloads are stored at 8 bits per channel like the
benchmark images (each value a multiple of 1/255 in [0, 1]).  Shapes follow the paper's workloads: 481x321 is the BSDS image
size (Sec. 5), the label counts lie in the Graz range of 2-13 labels and
the scribbles are painted with the Graz 13-pixel brush (Sec. 5.1).

The learned analysis operator of Sec. 2 is not available either; a seeded
Gaussian operator with zero-mean, unit-norm rows replaces it.

Nothing here evaluates any part of the method.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, Optional

import numpy as np

BASE_SEED = 13124746

# 8-neighbourhood used by the random-walk strokes (dx, dy).
_DIRS = np.array([(1, 0), (1, 1), (0, 1), (-1, 1), (-1, 0), (-1, -1), (0, -1), (1, -1)],
                 dtype=np.int64)


@dataclasses.dataclass
class Workload:
    """One synthetic problem instance.

    rgb:          float32 (3, H, W) colour planes (SoA), values roughly in [0, 1]
                  (with colour_levels n > 0: multiples of 1/n in [0, 1])
    omega:        float32 (k, n) analysis operator, n = p*p, row-major
    sample_pix:   int32 (M,) linear pixel index row*W + col of each scribble sample
    sample_label: int32 (M,) label of each sample, 0..L-1
    region:       int32 (H, W) ground-truth region index (label of each pixel)
    train_pix:    int32 (T,) pixels drawn for surrogate training (may be empty)
    """
    name: str
    H: int
    W: int
    p: int
    k: int
    L: int
    rgb: np.ndarray
    omega: np.ndarray
    sample_pix: np.ndarray
    sample_label: np.ndarray
    region: np.ndarray
    train_pix: np.ndarray
    mask_sigma: float
    sigma_c: float = 0.05
    alpha_rho: float = 1.3
    beta_scale: float = 1.0
    rho_floor_px: float = 1.0
    tau_frac: float = 0.1
    precision: str = "fp32"
    seed: int = 0
    colour_levels: int = 0

    @property
    def N(self) -> int:
        return self.H * self.W

    @property
    def n(self) -> int:
        return self.p * self.p

    @property
    def M(self) -> int:
        return int(self.sample_pix.shape[0])


# Shapes of the workloads: the tiny case, the BSDS-sized case and its BF16
# form, the large case and its BF16 form, and the surrogate case.
CONFIGS: Dict[int, dict] = {
    0: dict(name="tiny_64x64_p5_k50_L3", H=64, W=64, R=3, p=5, k=50,
            scribble="uniform", per_region=200, bandnoise=False, train_frac=0.0, colour_levels=255),
    1: dict(name="bsds_481x321_p7_k98_L10_fp32", H=321, W=481, R=10, p=7, k=98,
            scribble="strokes", total_frac=0.05, bandnoise=False, train_frac=0.0, colour_levels=255),
    2: dict(name="bsds_481x321_p7_k98_L10_bf16", H=321, W=481, R=10, p=7, k=98,
            scribble="strokes", total_frac=0.05, bandnoise=False, train_frac=0.0,
            precision="bf16", colour_levels=255),
    3: dict(name="large_1024x1024_p11_k242_L16", H=1024, W=1024, R=16, p=11, k=242,
            scribble="strokes", total=50000, bandnoise=True, train_frac=0.0, colour_levels=255),
    4: dict(name="surrogate_2048x2048_p7_k98_L10", H=2048, W=2048, R=10, p=7, k=98,
            scribble="strokes", total_frac=0.05, bandnoise=False, train_frac=0.02, colour_levels=255),
    5: dict(name="large_1024x1024_p11_k242_L16_bf16", H=1024, W=1024, R=16, p=11, k=242,
            scribble="strokes", total=50000, bandnoise=True, train_frac=0.0, precision="bf16",
            colour_levels=255),
}

# Precision forms run on exactly the inputs of their FP32 case.
_SAME_INPUTS = {2: 1, 5: 3}


def make_omega(k: int, n: int, rng: np.random.Generator) -> np.ndarray:
    """Seeded stand-in for the learned operator: N(0,1) rows, made zero-mean and
    then unit-norm in float64, rounded once to float32."""
    om = rng.standard_normal((k, n))
    om = om - om.mean(axis=1, keepdims=True)
    om = om / np.linalg.norm(om, axis=1, keepdims=True)
    return om.astype(np.float32)


def _voronoi(H: int, W: int, R: int, rng: np.random.Generator) -> np.ndarray:
    cx = rng.uniform(0.0, W, size=R)
    cy = rng.uniform(0.0, H, size=R)
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    best = np.full((H, W), np.inf)
    region = np.zeros((H, W), dtype=np.int32)
    for r in range(R):  # strict '<' keeps the lowest index on ties
        d = (xx - cx[r]) ** 2 + (yy - cy[r]) ** 2
        upd = d < best
        best[upd] = d[upd]
        region[upd] = r
    return region


def _image(region: np.ndarray, R: int, rng: np.random.Generator, bandnoise: bool,
           amp: float = 0.1, noise_sd: float = 0.05) -> np.ndarray:
    H, W = region.shape
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    img = np.zeros((3, H, W), dtype=np.float64)
    means = rng.uniform(0.0, 1.0, size=(R, 3))
    periods = rng.uniform(3.0, 12.0, size=R)
    thetas = rng.uniform(0.0, np.pi, size=R)
    phis = rng.uniform(0.0, 2.0 * np.pi, size=R)
    band_sigma = rng.uniform(1.0, 3.0, size=R) if bandnoise else None
    for r in range(R):
        sel = region == r
        tex = amp * np.sin(2.0 * np.pi * (xx[sel] * np.cos(thetas[r]) + yy[sel] * np.sin(thetas[r]))
                           / periods[r] + phis[r])
        if bandnoise:
            from scipy.ndimage import gaussian_filter
            white = rng.standard_normal((H, W))
            band = gaussian_filter(white, band_sigma[r], mode="reflect")
            band *= 0.05 / band.std()
            tex = tex + band[sel]
        for c in range(3):
            img[c][sel] = means[r, c] + tex
    img += rng.normal(0.0, noise_sd, size=img.shape)
    return img.astype(np.float32)


def quantise_colours(rgb: np.ndarray, n: int) -> np.ndarray:
    """Colours at n levels per channel: clipped to [0, 1], rounded to the
    nearest multiple of 1/n (float32 of q / n)."""
    q = np.rint(np.clip(rgb.astype(np.float64), 0.0, 1.0) * n)
    return (q / n).astype(np.float32)


def _split_targets(total: int, areas: np.ndarray) -> np.ndarray:
    """Integer shares proportional to area that sum exactly to `total`
    (largest-remainder rounding, ties to the lower region index)."""
    exact = total * areas / areas.sum()
    base = np.floor(exact).astype(np.int64)
    rem = total - int(base.sum())
    order = np.argsort(-(exact - base), kind="stable")
    base[order[:rem]] += 1
    return base


def _disc_offsets(diameter: int = 13):
    rad2 = (diameter / 2.0) ** 2
    h = diameter // 2
    offs = [(du, dv) for dv in range(-h, h + 1) for du in range(-h, h + 1) if du * du + dv * dv <= rad2]
    return np.array(offs, dtype=np.int64)


def _strokes(region: np.ndarray, r: int, target: int, rng: np.random.Generator,
             persistence: float = 0.7, stroke_len: int = 200, diameter: int = 13) -> np.ndarray:
    """Random-walk brush strokes inside region r, painted with a disc brush
    clipped to the region, truncated at exactly `target` distinct pixels."""
    H, W = region.shape
    inside = np.flatnonzero(region.ravel() == r)
    if target > inside.size:
        raise ValueError("region too small for its scribble share")
    taken = np.zeros(H * W, dtype=bool)
    out = []
    count = 0
    disc = _disc_offsets(diameter)
    while count < target:
        start = int(inside[rng.integers(inside.size)])
        cx, cy = start % W, start // W
        d = int(rng.integers(8))
        for _ in range(stroke_len):
            xs = cx + disc[:, 0]
            ys = cy + disc[:, 1]
            ok = (xs >= 0) & (xs < W) & (ys >= 0) & (ys < H)
            lin = ys[ok] * W + xs[ok]
            lin = lin[region.ravel()[lin] == r]
            lin = lin[~taken[lin]]
            if lin.size:
                lin = lin[: target - count]
                taken[lin] = True
                out.append(lin)
                count += lin.size
                if count >= target:
                    break
            if rng.random() >= persistence:
                d = int(rng.integers(8))
            nx, ny = cx + int(_DIRS[d, 0]), cy + int(_DIRS[d, 1])
            if 0 <= nx < W and 0 <= ny < H and region[ny, nx] == r:
                cx, cy = nx, ny
            else:
                d = int(rng.integers(8))
    return np.concatenate(out).astype(np.int32)


def make_workload(name: str, H: int, W: int, R: int, p: int, k: int, seed: int,
                  scribble: str = "uniform", per_region: int = 0, total: Optional[int] = None,
                  total_frac: Optional[float] = None, bandnoise: bool = False,
                  train_frac: float = 0.0, precision: str = "fp32",
                  mask_sigma: Optional[float] = None, colour_levels: int = 0) -> Workload:
    """Draw one workload.  Sub-streams (image, operator, scribbles, training
    pixels) are spawned from SeedSequence(seed) so each part is reproducible
    on its own.  colour_levels n > 0 stores the image at n levels per channel
    (clipped to [0, 1], rounded to the nearest multiple of 1/n)."""
    ss = np.random.SeedSequence(seed)
    s_img, s_om, s_scr, s_train, _s_mlp = ss.spawn(5)
    rng_img = np.random.default_rng(s_img)
    region = _voronoi(H, W, R, rng_img)
    rgb = _image(region, R, rng_img, bandnoise)
    if colour_levels > 0:
        rgb = quantise_colours(rgb, colour_levels)
    omega = make_omega(k, p * p, np.random.default_rng(s_om))

    rng_s = np.random.default_rng(s_scr)
    pix, lab = [], []
    if scribble == "uniform":
        for r in range(R):
            inside = np.flatnonzero(region.ravel() == r)
            take = min(per_region, inside.size)
            pix.append(rng_s.choice(inside, size=take, replace=False).astype(np.int32))
            lab.append(np.full(take, r, dtype=np.int32))
    elif scribble == "strokes":
        if total is None:
            total = int(np.floor(total_frac * H * W))
        areas = np.bincount(region.ravel(), minlength=R).astype(np.float64)
        targets = _split_targets(total, areas)
        for r in range(R):
            if targets[r] == 0:
                continue
            px = _strokes(region, r, int(targets[r]), rng_s)
            pix.append(px)
            lab.append(np.full(px.size, r, dtype=np.int32))
    else:
        raise ValueError(scribble)
    sample_pix = np.concatenate(pix).astype(np.int32)
    sample_label = np.concatenate(lab).astype(np.int32)

    if train_frac > 0:
        T = int(round(train_frac * H * W))
        train = np.random.default_rng(s_train).choice(H * W, size=T, replace=False)
        train_pix = np.sort(train).astype(np.int32)
    else:
        train_pix = np.zeros(0, dtype=np.int32)

    return Workload(name=name, H=H, W=W, p=p, k=k, L=R, rgb=rgb, omega=omega,
                    sample_pix=sample_pix, sample_label=sample_label, region=region,
                    train_pix=train_pix,
                    mask_sigma=(p / 4.0 if mask_sigma is None else mask_sigma),
                    precision=precision, seed=seed, colour_levels=colour_levels)


def make_config(c: int) -> Workload:
    """Workload c of CONFIGS with its fixed seed BASE_SEED + c.  The BF16
    precision forms (2 and 5) run on exactly the inputs of their FP32 cases
    (1 and 3)."""
    cfg = dict(CONFIGS[c])
    name = cfg.pop("name")
    seed = BASE_SEED + _SAME_INPUTS.get(c, c)
    return make_workload(name=name, seed=seed, **cfg)


def mlp_init(in_dim: int, hidden: int, out_dim: int, seed: int) -> np.ndarray:
    """Initial surrogate parameters (random numbers only), flat float32 in the
    order W1 (hidden x in_dim), b1, W2 (hidden x hidden), b2, W3 (out_dim x
    hidden), b3: each layer uniform in +-1/sqrt(fan_in)."""
    rng = np.random.default_rng(np.random.SeedSequence(seed))
    parts = []
    for fan_out, fan_in in ((hidden, in_dim), (hidden, hidden), (out_dim, hidden)):
        bound = 1.0 / np.sqrt(fan_in)
        parts.append(rng.uniform(-bound, bound, size=fan_out * fan_in))
        parts.append(rng.uniform(-bound, bound, size=fan_out))
    return np.concatenate(parts).astype(np.float32)


def mlp_order(n_rows: int, steps: int, batch: int, seed: int) -> np.ndarray:
    """Data order of `steps` batches: consecutive epochs, each a fresh random
    permutation of the rows (int32, steps x batch)."""
    rng = np.random.default_rng(np.random.SeedSequence(seed))
    need = steps * batch
    chunks, have = [], 0
    while have < need:
        chunks.append(rng.permutation(n_rows))
        have += n_rows
    return np.concatenate(chunks)[:need].astype(np.int32).reshape(steps, batch)


def unsup_init(N: int, colour_classes: int, texture_classes: int, seed: int):
    """Pixels whose colours and co-supports start the unsupervised clustering
    (random numbers only): distinct pixels drawn uniformly."""
    rng = np.random.default_rng(np.random.SeedSequence(seed))
    pix = rng.choice(N, size=colour_classes + texture_classes, replace=False).astype(np.int32)
    return pix[:colour_classes], pix[colour_classes:]
