"""FP64 oracle of the learned surrogate of the data term.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark may import this module; the product library never does.

The surrogate is a two-hidden-layer perceptron that maps a pixel's colour,
normalised position and analysed vector to its per-label log-likelihoods
(the data term of Sec. 3.2, computed exactly by the Parzen sum of Sec. 3.1,
is its training target).  The paper does not describe a surrogate; the
architecture, loss and optimiser below are the readings fixed for it:

* input x = [r, g, b, col/(W-1), row/(H-1), a_0 .. a_{k-1}]
  (a zero position coordinate when the image is one pixel wide or high);
* z1 = W1 x + b1, h1 = GELU(z1); z2 = W2 h1 + b2, h2 = GELU(z2);
  y = W3 h2 + b3, with the exact (erf) GELU(z) = z Phi(z);
* loss = mean over the batch and the labels of (y - t)^2 with the clipped
  target t_i = max(l_i, max_j l_j - 20);
* Adam (beta1 0.9, beta2 0.999, eps 1e-8) with bias correction.

Parameters travel as one flat FP32/FP64 vector in the order
W1 (hidden x in, row-major), b1, W2 (hidden x hidden), b2, W3 (out x hidden), b3.

``emulate_bf16`` rounds the operands of every matrix product to BF16
(round to nearest even, via FP32) at exactly the points where the GPU does:
the layer inputs and weights of the forward products, the output delta and
the hidden deltas with the transposed weights in the backward products, and
both operands of the weight-gradient products.  Everything else stays FP64.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
from scipy.special import erf

CLIP_NATS = 20.0
ADAM_B1, ADAM_B2, ADAM_EPS = 0.9, 0.999, 1e-8


def round_bf16(x) -> np.ndarray:
    """FP64 -> FP32 (nearest) -> BF16 (nearest, ties to even), returned as FP64."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    u = (u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)
    nan = np.isnan(f)
    out = u.astype(np.uint32).view(np.float32).astype(np.float64)
    out[nan] = np.nan
    return out


def gelu(z: np.ndarray) -> np.ndarray:
    """GELU(z) = z * Phi(z), Phi the standard normal CDF."""
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z: np.ndarray) -> np.ndarray:
    """d GELU / dz = Phi(z) + z phi(z)."""
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


@dataclass
class Shapes:
    n_in: int
    hidden: int
    n_out: int

    @property
    def sizes(self):
        h, i, o = self.hidden, self.n_in, self.n_out
        return [("W1", (h, i)), ("b1", (h,)), ("W2", (h, h)), ("b2", (h,)), ("W3", (o, h)), ("b3", (o,))]

    @property
    def count(self) -> int:
        return sum(int(np.prod(s)) for _, s in self.sizes)


def unpack(flat: np.ndarray, sh: Shapes) -> dict:
    out, off = {}, 0
    for name, shape in sh.sizes:
        n = int(np.prod(shape))
        out[name] = np.asarray(flat[off:off + n], dtype=np.float64).reshape(shape)
        off += n
    assert off == flat.size
    return out


def pack(parts: dict, sh: Shapes) -> np.ndarray:
    return np.concatenate([np.asarray(parts[name], np.float64).ravel() for name, _ in sh.sizes])


def features(rgb: np.ndarray, alpha: np.ndarray, pix: np.ndarray) -> np.ndarray:
    """Surrogate inputs of the pixels `pix` (linear indices): colour, position
    normalised to [0, 1] and the analysed vector."""
    _, H, W = rgb.shape
    pix = np.asarray(pix, np.int64)
    r, c = pix // W, pix % W
    flat = rgb.reshape(3, -1).astype(np.float64)
    cols = [flat[0, pix], flat[1, pix], flat[2, pix],
            c / (W - 1) if W > 1 else np.zeros(len(pix)),
            r / (H - 1) if H > 1 else np.zeros(len(pix))]
    a = np.asarray(alpha, np.float64).reshape(H * W, -1)[pix]
    return np.concatenate([np.stack(cols, 1), a], 1)


def clip_targets(ell: np.ndarray) -> np.ndarray:
    """t_i = max(l_i, max_j l_j - 20) per pixel (row)."""
    ell = np.asarray(ell, np.float64)
    return np.maximum(ell, ell.max(1, keepdims=True) - CLIP_NATS)


def forward(flat: np.ndarray, sh: Shapes, X: np.ndarray, emulate_bf16: bool = False) -> dict:
    p = unpack(flat, sh)
    q = round_bf16 if emulate_bf16 else (lambda v: np.asarray(v, np.float64))
    X = np.asarray(X, np.float64)
    z1 = q(X) @ q(p["W1"]).T + p["b1"]
    h1 = gelu(z1)
    z2 = q(h1) @ q(p["W2"]).T + p["b2"]
    h2 = gelu(z2)
    y = q(h2) @ q(p["W3"]).T + p["b3"]
    return {"X": X, "z1": z1, "h1": h1, "z2": z2, "h2": h2, "y": y}


def loss_and_grad(flat: np.ndarray, sh: Shapes, X: np.ndarray, T: np.ndarray,
                  emulate_bf16: bool = False):
    """Mean squared error over batch and labels, and its gradient (flat)."""
    p = unpack(flat, sh)
    q = round_bf16 if emulate_bf16 else (lambda v: np.asarray(v, np.float64))
    f = forward(flat, sh, X, emulate_bf16)
    B, L = f["y"].shape
    d = f["y"] - np.asarray(T, np.float64)
    loss = float((d * d).sum() / (B * L))
    dy = 2.0 * d / (B * L)
    dh2 = q(dy) @ q(p["W3"])
    dz2 = dh2 * gelu_grad(f["z2"])
    dh1 = q(dz2) @ q(p["W2"])
    dz1 = dh1 * gelu_grad(f["z1"])
    g = {
        "W3": q(dy).T @ q(f["h2"]), "b3": dy.sum(0),
        "W2": q(dz2).T @ q(f["h1"]), "b2": dz2.sum(0),
        "W1": q(dz1).T @ q(f["X"]), "b1": dz1.sum(0),
    }
    return loss, pack(g, sh)


def adam_step(flat: np.ndarray, grad: np.ndarray, m: np.ndarray, v: np.ndarray, t: int, lr: float):
    """One Adam update (step number t >= 1); returns (params, m, v)."""
    m = ADAM_B1 * m + (1.0 - ADAM_B1) * grad
    v = ADAM_B2 * v + (1.0 - ADAM_B2) * grad * grad
    mhat = m / (1.0 - ADAM_B1 ** t)
    vhat = v / (1.0 - ADAM_B2 ** t)
    return flat - lr * mhat / (np.sqrt(vhat) + ADAM_EPS), m, v


def train(flat0: np.ndarray, sh: Shapes, X: np.ndarray, T: np.ndarray, order: np.ndarray,
          lr: float = 1e-3, emulate_bf16: bool = False):
    """Adam over the batches order[s] (row indices into X, T), one step each.
    Returns the parameters and the loss of every step (before its update)."""
    flat = np.asarray(flat0, np.float64).copy()
    m = np.zeros_like(flat)
    v = np.zeros_like(flat)
    losses = []
    for s, idx in enumerate(np.asarray(order)):
        loss, g = loss_and_grad(flat, sh, X[idx], T[idx], emulate_bf16)
        losses.append(loss)
        flat, m, v = adam_step(flat, g, m, v, s + 1, lr)
    return flat, np.asarray(losses)


def argmax_labels(ell: np.ndarray) -> np.ndarray:
    """Label decision per pixel; ties go to the lowest label index."""
    return np.argmax(np.asarray(ell), axis=1)
