"""FP64 CPU oracle of the co-sparse data term (ctypes wrapper).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this package; the product library never
does.  The arithmetic lives in ``cso_oracle.c`` (plain C, FP64, no FMA
contraction); this wrapper only marshals numpy arrays.  ``build()`` compiles
the shared library with gcc; ``lib()`` builds it on first use when missing.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cso_oracle.c")
_SO = os.path.join(_HERE, "libcso_oracle.so")

CSO_OK = 0
CSO_ERR_ARG = 1
CSO_ERR_EMPTY_LABEL = 2
CSO_ERR_NOMEM = 4
CSO_ERR_NONFINITE = 5

_lib = None


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what} failed with oracle status {code}")
        self.code = code


def build(force: bool = True) -> str:
    """Compile the oracle: gcc -O2 -ffp-contract=off -fopenmp (IEEE double,
    no FMA contraction, no fast-math)."""
    if not force and os.path.exists(_SO) and os.path.getmtime(_SO) >= os.path.getmtime(_SRC):
        return _SO
    tmp = _SO + f".tmp{os.getpid()}"
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
           "-std=c11", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True, cwd=_HERE)
    os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO):
        build(force=True)
    L = ctypes.CDLL(_SO)
    P = ctypes.c_void_p
    i32, i64, dbl = ctypes.c_int, ctypes.c_int64, ctypes.c_double
    sigs = {
        "cso_set_threads": (None, [i32]),
        "cso_get_threads": (i32, []),
        "cso_gray": (i32, [P, i32, i32, P]),
        "cso_mask_table": (i32, [i32, dbl, P]),
        "cso_patches": (i32, [P, i32, i32, i32, dbl, P, i64, P]),
        "cso_analyze": (i32, [P, i32, i32, i32, dbl, P, i32, P, i64, P]),
        "cso_tau_median": (i32, [P, i64, dbl, P, P]),
        "cso_cosupport": (i32, [P, i64, i32, dbl, P]),
        "cso_tsm": (i32, [P, i64, P, i64, i32, P]),
        "cso_nearest_d2": (i32, [i32, i32, P, P, i64, i32, P, i64, P]),
        "cso_label_loglik": (i32, [P, i32, i32, P, i32, P, P, i64, i32, dbl, dbl, dbl, dbl, i32,
                                   P, i64, P]),
        "cso_label_rep": (i32, [P, i64, i32, P, P, i64, i32, P]),
        "cso_label_rep_soft": (i32, [P, i64, i32, dbl, P, P, i64, i32, P]),
        "cso_label_loglik_soft": (i32, [P, i32, i32, P, i32, dbl, P, P, i64, i32, dbl, dbl, dbl,
                                        dbl, i32, P, i64, P]),
        "cso_label_loglik_joint": (i32, [P, i32, i32, P, i32, P, P, i64, i32, dbl, dbl, dbl, dbl,
                                         i32, P, i64, P]),
    }
    for name, (res, args) in sigs.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


def _check(code: int, what: str):
    if code != CSO_OK:
        raise OracleError(code, what)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def set_threads(n: int) -> None:
    lib().cso_set_threads(int(n))


def get_threads() -> int:
    return int(lib().cso_get_threads())


def gray(rgb: np.ndarray) -> np.ndarray:
    rgb = _c(rgb, np.float32)
    _, H, W = rgb.shape
    out = np.empty((H, W), dtype=np.float64)
    _check(lib().cso_gray(_p(rgb), H, W, _p(out)), "cso_gray")
    return out


def mask_table(p: int, sigma: float) -> np.ndarray:
    out = np.empty((p, p), dtype=np.float64)
    _check(lib().cso_mask_table(p, float(sigma), _p(out)), "cso_mask_table")
    return out


def patches(rgb, p: int, mask_sigma: float, pix=None) -> np.ndarray:
    rgb = _c(rgb, np.float32)
    _, H, W = rgb.shape
    pix_a = None if pix is None else _c(pix, np.int32)
    cnt = H * W if pix_a is None else pix_a.size
    out = np.empty((cnt, p * p), dtype=np.float64)
    _check(lib().cso_patches(_p(rgb), H, W, p, float(mask_sigma), _p(pix_a), cnt, _p(out)),
           "cso_patches")
    return out


def analyze(rgb, p: int, mask_sigma: float, omega, pix=None) -> np.ndarray:
    rgb = _c(rgb, np.float32)
    omega = _c(omega, np.float32)
    _, H, W = rgb.shape
    k = omega.shape[0]
    pix_a = None if pix is None else _c(pix, np.int32)
    cnt = H * W if pix_a is None else pix_a.size
    out = np.empty((cnt, k), dtype=np.float64)
    _check(lib().cso_analyze(_p(rgb), H, W, p, float(mask_sigma), _p(omega), k, _p(pix_a), cnt,
                             _p(out)), "cso_analyze")
    return out


def tau_median(alpha: np.ndarray, frac: float = 0.1):
    """Returns (tau, median)."""
    a = _c(alpha, np.float64).ravel()
    tau = ctypes.c_double()
    med = ctypes.c_double()
    _check(lib().cso_tau_median(_p(a), a.size, float(frac), ctypes.byref(tau), ctypes.byref(med)),
           "cso_tau_median")
    return tau.value, med.value


def cosupport(alpha: np.ndarray, tau: float) -> np.ndarray:
    a = _c(alpha, np.float64)
    npix, k = a.shape
    out = np.empty((npix, (k + 63) // 64), dtype=np.uint64)
    _check(lib().cso_cosupport(_p(a), npix, k, float(tau), _p(out)), "cso_cosupport")
    return out


def tsm(A: np.ndarray, B: np.ndarray, k: int) -> np.ndarray:
    A = _c(A, np.uint64)
    B = _c(B, np.uint64)
    na, nb = A.shape[0], B.shape[0]
    out = np.empty((na, nb), dtype=np.int32)
    _check(lib().cso_tsm(_p(A), na, _p(B), nb, k, _p(out)), "cso_tsm")
    return out


def nearest_d2(H: int, W: int, sample_pix, sample_label, L: int, pix=None) -> np.ndarray:
    sp = _c(sample_pix, np.int32)
    sl = _c(sample_label, np.int32)
    pix_a = None if pix is None else _c(pix, np.int32)
    cnt = H * W if pix_a is None else pix_a.size
    out = np.empty((cnt, L), dtype=np.int64)
    _check(lib().cso_nearest_d2(H, W, _p(sp), _p(sl), sp.size, L, _p(pix_a), cnt, _p(out)),
           "cso_nearest_d2")
    return out


def label_rep(masks, k: int, sample_pix, sample_label, L: int) -> np.ndarray:
    """Textural representative c_i of every label (majority of its samples'
    co-supports): L x ceil(k/64) uint64."""
    masks = _c(masks, np.uint64)
    sp = _c(sample_pix, np.int32)
    sl = _c(sample_label, np.int32)
    out = np.empty((L, (k + 63) // 64), dtype=np.uint64)
    _check(lib().cso_label_rep(_p(masks), masks.shape[0], k, _p(sp), _p(sl), sp.size, L, _p(out)),
           "cso_label_rep")
    return out


def label_rep_soft(alpha, sigma_iota: float, sample_pix, sample_label, L: int) -> np.ndarray:
    """Median representative of the smooth co-supports of every label: L x k."""
    a = _c(alpha, np.float64)
    sp = _c(sample_pix, np.int32)
    sl = _c(sample_label, np.int32)
    out = np.empty((L, a.shape[1]), dtype=np.float64)
    _check(lib().cso_label_rep_soft(_p(a), a.shape[0], a.shape[1], float(sigma_iota), _p(sp), _p(sl),
                                    sp.size, L, _p(out)), "cso_label_rep_soft")
    return out


def label_loglik_soft(rgb, alpha, sigma_iota: float, sample_pix, sample_label, L: int,
                      alpha_rho: float = 1.3, sigma_c: float = 0.05, beta_scale: float = 1.0,
                      rho_floor: float = 1.0, normalise: bool = False, pix=None) -> np.ndarray:
    """Joint form with smooth co-supports (eq:map_tsm, eq:tsm, eq:approx_cosupp)."""
    rgb = _c(rgb, np.float32)
    _, H, W = rgb.shape
    a = _c(alpha, np.float64)
    sp = _c(sample_pix, np.int32)
    sl = _c(sample_label, np.int32)
    pix_a = None if pix is None else _c(pix, np.int32)
    cnt = H * W if pix_a is None else pix_a.size
    out = np.empty((cnt, L), dtype=np.float64)
    _check(lib().cso_label_loglik_soft(_p(rgb), H, W, _p(a), a.shape[1], float(sigma_iota), _p(sp),
                                       _p(sl), sp.size, L, float(alpha_rho), float(sigma_c),
                                       float(beta_scale), float(rho_floor), int(bool(normalise)),
                                       _p(pix_a), cnt, _p(out)), "cso_label_loglik_soft")
    return out


def label_loglik(rgb, masks, k: int, sample_pix, sample_label, L: int, alpha_rho: float = 1.3,
                 sigma_c: float = 0.05, beta_scale: float = 1.0, rho_floor: float = 1.0,
                 normalise: bool = False, pix=None, joint: bool = False) -> np.ndarray:
    """joint=False: texture factor per sample inside the Parzen sum;
    joint=True: colour/location Parzen density times the texture posterior
    against the label representatives (eq:joined)."""
    rgb = _c(rgb, np.float32)
    _, H, W = rgb.shape
    masks = _c(masks, np.uint64)
    sp = _c(sample_pix, np.int32)
    sl = _c(sample_label, np.int32)
    pix_a = None if pix is None else _c(pix, np.int32)
    cnt = H * W if pix_a is None else pix_a.size
    out = np.empty((cnt, L), dtype=np.float64)
    fn = lib().cso_label_loglik_joint if joint else lib().cso_label_loglik
    _check(fn(_p(rgb), H, W, _p(masks), k, _p(sp), _p(sl), sp.size, L,
              float(alpha_rho), float(sigma_c), float(beta_scale),
              float(rho_floor), int(bool(normalise)), _p(pix_a), cnt, _p(out)),
           "cso_label_loglik")
    return out


def full_masks(w, tau=None):
    """Masks of every pixel of workload w via the oracle's own steps; returns
    (masks, tau, alpha)."""
    alpha = analyze(w.rgb, w.p, w.mask_sigma, w.omega)
    if tau is None:
        tau, _ = tau_median(alpha, w.tau_frac)
    return cosupport(alpha, tau), tau, alpha
