"""ctypes binding of libcosparse.so.  Argument marshalling only."""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import Optional

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.environ.get("COSPARSE_LIBRARY") or os.path.join(_HERE, "libcosparse.so")

CS_OK = 0
CS_ERR_ARG = 1
CS_ERR_EMPTY_LABEL = 2
CS_ERR_HIP = 3
CS_ERR_NOMEM = 4
CS_ERR_NONFINITE = 5
CS_FP32 = 0
CS_BF16 = 1
CS_FP64 = 2

_PREC = {"fp32": CS_FP32, "bf16": CS_BF16, "fp64": CS_FP64, CS_FP32: CS_FP32, CS_BF16: CS_BF16, CS_FP64: CS_FP64}

# Every entry point the header declares, with (restype, argtypes).
_P, _I, _I64, _D = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double


class _LoglikParamsC(ctypes.Structure):
    _fields_ = [("alpha_rho", ctypes.c_double), ("sigma_c", ctypes.c_double),
                ("beta_scale", ctypes.c_double), ("rho_floor_px", ctypes.c_double),
                ("normalise", ctypes.c_int), ("colour_levels", ctypes.c_int)]


class _LoglikStatsC(ctypes.Structure):
    _fields_ = [("rescaled_chunks", ctypes.c_int64), ("overflow_tiles", ctypes.c_int64),
                ("exact_tiles", ctypes.c_int64)]


class _SegmentParamsC(ctypes.Structure):
    _fields_ = [("lambda_", ctypes.c_double), ("gamma", ctypes.c_double), ("nu", ctypes.c_double),
                ("iterations", ctypes.c_int), ("precision", ctypes.c_int)]


class _SegmentStatsC(ctypes.Structure):
    _fields_ = [("primal", ctypes.c_double), ("binary", ctypes.c_double), ("dual", ctypes.c_double),
                ("gamma", ctypes.c_double), ("labels_used", ctypes.c_int)]


class _UnsupParamsC(ctypes.Structure):
    _fields_ = [("colour_classes", ctypes.c_int), ("texture_classes", ctypes.c_int), ("iterations", ctypes.c_int),
                ("sigma_c", ctypes.c_double), ("beta", ctypes.c_double)]


class _CosupportStatsC(ctypes.Structure):
    _fields_ = [("recomputed", ctypes.c_int64), ("max_margin", ctypes.c_double)]


SIGNATURES = {
    "cs_create": (_I, [ctypes.POINTER(_P), _I, _P]),
    "cs_destroy": (_I, [_P]),
    "cs_set_stream": (_I, [_P, _P]),
    "cs_last_error": (ctypes.c_char_p, [_P]),
    "cs_set_check_finite": (_I, [_P, _I]),
    "cs_analyze_patches": (_I, [_P, _P, _I, _I, _I, _D, _P, _I, _I, _P]),
    "cs_tau_median": (_I, [_P, _P, _I, _I, _I, _D, _P, _I, _I, _P, _D, ctypes.POINTER(_D)]),
    "cs_cosupport": (_I, [_P, _P, _I, _I, _I, _D, _P, _I, _I, _P, _D, _D, _P,
                          ctypes.POINTER(_CosupportStatsC)]),
    "cs_cosupport_noalloc": (_I, [_P, _P, _I, _I, _I, _D, _P, _I, _I, _P, _D, _D, _P]),
    "cs_cosupport_median": (_I, [_P, _P, _I, _I, _I, _D, _P, _I, _I, _D, _D, _P, _P, _P]),
    "cs_texture_similarity": (_I, [_P, _P, _I64, _P, _I64, _I, _P]),
    "cs_label_loglik": (_I, [_P, _P, _I, _I, _P, _I, _P, _P, _I64, _I,
                             ctypes.POINTER(_LoglikParamsC), _P, _I64, _P]),
    "cs_label_loglik_joint": (_I, [_P, _P, _I, _I, _P, _I, _P, _P, _I64, _I,
                                   ctypes.POINTER(_LoglikParamsC), _P, _I64, _P]),
    "cs_label_loglik_soft": (_I, [_P, _P, _I, _I, _P, _I, _D, _P, _P, _I64, _I,
                                  ctypes.POINTER(_LoglikParamsC), _P, _I64, _P]),
    "cs_last_loglik_stats": (_I, [_P, ctypes.POINTER(_LoglikStatsC)]),
    "cs_profile_enable": (_I, [_P, _I]),
    "cs_profile_only": (_I, [_P, ctypes.c_char_p]),
    "cs_profile_sample": (_I, [_P, ctypes.c_int]),
    "cs_profile_read": (_I, [_P, ctypes.c_char_p, ctypes.POINTER(_D), ctypes.POINTER(_I64)]),
    "cs_edge_weight": (_I, [_P, _P, _I, _I, _D, _P, ctypes.POINTER(_D)]),
    "cs_segment": (_I, [_P, _P, _I, _I, _P, _I, ctypes.POINTER(_SegmentParamsC), _P, _P,
                        ctypes.POINTER(_SegmentStatsC)]),
    "cs_unsupervised_loglik": (_I, [_P, _P, _I, _I, _P, _I, _P, _P, ctypes.POINTER(_UnsupParamsC), _P, _P, _P,
                                    _P, _P]),
    "cs_mlp_param_count": (_I64, [_I, _I, _I]),
    "cs_mlp_init": (_I, [_P, ctypes.POINTER(_P), _I, _I, _I, _P]),
    "cs_mlp_free": (_I, [_P]),
    "cs_mlp_get_params": (_I, [_P, _P, _P]),
    "cs_mlp_features": (_I, [_P, _P, _I, _I, _P, _I, _P, _I64, _P]),
    "cs_mlp_grad": (_I, [_P, _P, _P, _P, _I64, _P, _P]),
    "cs_mlp_train": (_I, [_P, _P, _P, _P, _I64, _P, _I64, _I, _D, _P]),
    "cs_mlp_fit_output_bias": (_I, [_P, _P, _P, _I64]),
    "cs_mlp_infer": (_I, [_P, _P, _P, _I, _I, _P, _I, _P]),
    "cs_mlp_forward": (_I, [_P, _P, _P, _I64, _P]),
    "cs_mlp_infer_fallback": (_I, [_P, _P, _P, _I, _I, _P, _I, _P, _I, _P, _P, _I64, _I,
                                   ctypes.POINTER(_LoglikParamsC), _D, _P, ctypes.POINTER(_I64)]),
}

_lib = None


class CosparseError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"cosparse error {code}: {msg}")
        self.code = code


def library_path() -> str:
    return _SO


def lib():
    """Load libcosparse.so; raises when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO):
        raise RuntimeError(f"{_SO} is missing: build it with __graft_entry__.build() "
                           "(python paper_1312_4746_amd/build.py)")
    L = ctypes.CDLL(_SO)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _nw(k: int) -> int:
    return (int(k) + 63) // 64


def _image_hw(rgb) -> tuple:
    """(H, W) of a (3, H, W) colour tensor."""
    if rgb.dim() != 3 or rgb.shape[0] != 3:
        raise ValueError(f"rgb must be (3, H, W), got {tuple(rgb.shape)}")
    return int(rgb.shape[1]), int(rgb.shape[2])


def _omega_k(omega, p: int) -> int:
    if omega.dim() != 2 or omega.shape[1] != p * p:
        raise ValueError(f"omega must be (k, p*p) = (k, {p * p}), got {tuple(omega.shape)}")
    return int(omega.shape[0])


def _numel(t, n: int, name: str, what: str):
    """The device kernels see only pointers: a buffer of the wrong size would be
    read or written out of bounds, so sizes are checked before any launch."""
    if t is not None and t.numel() != n:
        raise ValueError(f"{name} must hold {what} = {n} elements, got {t.numel()}")


def _masks_shape(masks, npix: int, k: int, name: str = "masks"):
    if masks.dim() != 2 or masks.shape[0] != npix or masks.shape[1] != _nw(k):
        raise ValueError(f"{name} must be (N, ceil(k/64)) = ({npix}, {_nw(k)}), got {tuple(masks.shape)}")


def _samples(sample_pix, sample_label):
    if sample_label.numel() != sample_pix.numel():
        raise ValueError(f"sample_label holds {sample_label.numel()} labels for {sample_pix.numel()} samples")


@dataclasses.dataclass
class LoglikParams:
    alpha_rho: float = 1.3
    sigma_c: float = 0.05
    beta_scale: float = 1.0
    rho_floor_px: float = 1.0
    normalise: bool = False
    # 0: colours are any floats; n in 1..255: every colour value is a multiple
    # of 1/n (255 for 8-bit images)
    colour_levels: int = 0

    def c(self) -> _LoglikParamsC:
        return _LoglikParamsC(self.alpha_rho, self.sigma_c, self.beta_scale, self.rho_floor_px,
                              int(bool(self.normalise)), int(self.colour_levels))


@dataclasses.dataclass
class UnsupParams:
    colour_classes: int = 4
    texture_classes: int = 4
    iterations: int = 10
    sigma_c: float = 0.05
    beta: float = 2.0

    def c(self) -> _UnsupParamsC:
        return _UnsupParamsC(int(self.colour_classes), int(self.texture_classes), int(self.iterations),
                             float(self.sigma_c), float(self.beta))


@dataclasses.dataclass
class SegmentParams:
    lam: float = 1.0
    gamma: float = 0.0
    nu: float = 0.0
    iterations: int = 300
    precision: str = "fp32"

    def c(self) -> _SegmentParamsC:
        return _SegmentParamsC(float(self.lam), float(self.gamma), float(self.nu), int(self.iterations),
                               _PREC[self.precision])


class Context:
    """One library context on one device; calls enqueue on torch's current
    stream of that device."""

    def __init__(self, device: int = 0):
        self.device = device
        self._h = ctypes.c_void_p()
        stream = torch.cuda.current_stream(device).cuda_stream
        rc = lib().cs_create(ctypes.byref(self._h), device, ctypes.c_void_p(stream))
        if rc != CS_OK:
            raise CosparseError(rc, "cs_create failed")

    def close(self):
        if self._h:
            lib().cs_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- helpers --------------------------------------------------------
    def _sync_stream(self):
        lib().cs_set_stream(self._h, ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream))

    def _check(self, rc: int):
        if rc != CS_OK:
            raise CosparseError(rc, lib().cs_last_error(self._h).decode())

    def _dev(self, t: torch.Tensor, dtype, name: str) -> torch.Tensor:
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise TypeError(f"{name} must be a device tensor")
        if t.dtype != dtype:
            raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        return t

    # -- C-ABI calls ----------------------------------------------------
    def analyze_patches(self, rgb: torch.Tensor, p: int, mask_sigma: float, omega: torch.Tensor,
                        precision="fp32", out: Optional[torch.Tensor] = None) -> torch.Tensor:
        H, W = _image_hw(rgb)
        k = _omega_k(omega, p)
        _numel(out, H * W * k, "alpha", "H*W*k")
        self._dev(rgb, torch.float32, "rgb")
        self._dev(omega, torch.float32, "omega")
        if out is None:
            out = torch.empty((H * W, k), dtype=torch.float32, device=rgb.device)
        self._dev(out, torch.float32, "alpha")
        self._sync_stream()
        self._check(lib().cs_analyze_patches(self._h, _ptr(rgb), H, W, p, float(mask_sigma),
                                             _ptr(omega), k, _PREC[precision], _ptr(out)))
        return out

    def tau_median(self, rgb, p, mask_sigma, omega, alpha, frac=0.1, precision="fp32") -> float:
        H, W = _image_hw(rgb)
        k = _omega_k(omega, p)
        _numel(alpha, H * W * k, "alpha", "H*W*k")
        self._dev(rgb, torch.float32, "rgb")
        self._dev(omega, torch.float32, "omega")
        self._dev(alpha, torch.float32, "alpha")
        tau = ctypes.c_double()
        self._sync_stream()
        self._check(lib().cs_tau_median(self._h, _ptr(rgb), H, W, p, float(mask_sigma), _ptr(omega),
                                        k, _PREC[precision], _ptr(alpha), float(frac),
                                        ctypes.byref(tau)))
        return tau.value

    def cosupport(self, rgb, p, mask_sigma, omega, tau, margin=-1.0, precision="fp32",
                  out: Optional[torch.Tensor] = None, stats: bool = False,
                  alpha: Optional[torch.Tensor] = None):
        """Masks as an int64 tensor (N, ceil(k/64)) holding the uint64 bit
        patterns; with stats=True returns (masks, {recomputed, max_margin}).
        With alpha (the analysed vectors of the same inputs and precision) the
        masks are decided from it instead of a fresh analysis."""
        H, W = _image_hw(rgb)
        k = _omega_k(omega, p)
        _numel(alpha, H * W * k, "alpha", "H*W*k")
        if out is not None:
            _masks_shape(out, H * W, k)
        self._dev(rgb, torch.float32, "rgb")
        self._dev(omega, torch.float32, "omega")
        if alpha is not None:
            self._dev(alpha, torch.float32, "alpha")
        if out is None:
            out = torch.empty((H * W, (k + 63) // 64), dtype=torch.int64, device=rgb.device)
        self._dev(out, torch.int64, "masks")
        st = _CosupportStatsC()
        self._sync_stream()
        self._check(lib().cs_cosupport(self._h, _ptr(rgb), H, W, p, float(mask_sigma), _ptr(omega),
                                       k, _PREC[precision], _ptr(alpha) if alpha is not None else None,
                                       float(tau), float(margin), _ptr(out),
                                       ctypes.byref(st) if stats else None))
        if stats:
            return out, {"recomputed": int(st.recomputed), "max_margin": float(st.max_margin)}
        return out

    def cosupport_noalloc(self, rgb, p, mask_sigma, omega, tau, out: torch.Tensor, margin=-1.0,
                          precision="fp32", alpha: Optional[torch.Tensor] = None) -> torch.Tensor:
        """cs_cosupport_noalloc: the masks of cosupport() from a call that
        allocates nothing (the caller passes the output buffer)."""
        H, W = _image_hw(rgb)
        k = _omega_k(omega, p)
        _numel(alpha, H * W * k, "alpha", "H*W*k")
        _masks_shape(out, H * W, k)
        self._dev(rgb, torch.float32, "rgb")
        self._dev(omega, torch.float32, "omega")
        if alpha is not None:
            self._dev(alpha, torch.float32, "alpha")
        self._dev(out, torch.int64, "masks")
        self._sync_stream()
        self._check(lib().cs_cosupport_noalloc(self._h, _ptr(rgb), H, W, p, float(mask_sigma), _ptr(omega), k,
                                               _PREC[precision], _ptr(alpha), float(tau), float(margin),
                                               _ptr(out)))
        return out

    def cosupport_median(self, rgb, p, mask_sigma, omega, frac=0.1, margin=-1.0, precision="fp32",
                         alpha: Optional[torch.Tensor] = None, out: Optional[torch.Tensor] = None,
                         tau: Optional[torch.Tensor] = None):
        """Analysed vectors, tau = frac * median|a| and the masks at that tau
        in one enqueue-only call.  Returns (alpha (N, k) float32, masks (N,
        ceil(k/64)) int64, tau (1,) float64 on the device)."""
        H, W = _image_hw(rgb)
        k = _omega_k(omega, p)
        _numel(alpha, H * W * k, "alpha", "H*W*k")
        if out is not None:
            _masks_shape(out, H * W, k)
        _numel(tau, 1, "tau", "one value")
        self._dev(rgb, torch.float32, "rgb")
        self._dev(omega, torch.float32, "omega")
        if alpha is None:
            alpha = torch.empty((H * W, k), dtype=torch.float32, device=rgb.device)
        self._dev(alpha, torch.float32, "alpha")
        if out is None:
            out = torch.empty((H * W, (k + 63) // 64), dtype=torch.int64, device=rgb.device)
        self._dev(out, torch.int64, "masks")
        if tau is None:
            tau = torch.empty(1, dtype=torch.float64, device=rgb.device)
        self._dev(tau, torch.float64, "tau")
        self._sync_stream()
        self._check(lib().cs_cosupport_median(self._h, _ptr(rgb), H, W, p, float(mask_sigma), _ptr(omega), k,
                                              _PREC[precision], float(frac), float(margin), _ptr(alpha),
                                              _ptr(out), _ptr(tau)))
        return alpha, out, tau

    def texture_similarity(self, A: torch.Tensor, B: torch.Tensor, k: int,
                           out: Optional[torch.Tensor] = None) -> torch.Tensor:
        _masks_shape(A, A.shape[0] if A.dim() == 2 else -1, k, "A")
        _masks_shape(B, B.shape[0] if B.dim() == 2 else -1, k, "B")
        na, nb = A.shape[0], B.shape[0]
        _numel(out, na * nb, "out", "na*nb")
        self._dev(A, torch.int64, "A")
        self._dev(B, torch.int64, "B")
        if out is None:
            out = torch.empty((na, nb), dtype=torch.int32, device=A.device)
        self._dev(out, torch.int32, "out")
        self._sync_stream()
        self._check(lib().cs_texture_similarity(self._h, _ptr(A), na, _ptr(B), nb, k, _ptr(out)))
        return out

    def label_loglik(self, rgb, masks, k: int, sample_pix, sample_label, L: int,
                     params: Optional[LoglikParams] = None, pix_subset=None,
                     out: Optional[torch.Tensor] = None, joint: bool = False) -> torch.Tensor:
        """joint=False: cs_label_loglik (texture factor per sample inside the
        Parzen sum); joint=True: cs_label_loglik_joint (eq:joined)."""
        H, W = _image_hw(rgb)
        _masks_shape(masks, H * W, k)
        _samples(sample_pix, sample_label)
        npix = H * W if pix_subset is None else pix_subset.numel()
        _numel(out, npix * L, "loglik", "npix*L")
        self._dev(rgb, torch.float32, "rgb")
        self._dev(masks, torch.int64, "masks")
        self._dev(sample_pix, torch.int32, "sample_pix")
        self._dev(sample_label, torch.int32, "sample_label")
        params = params or LoglikParams()
        if pix_subset is not None:
            self._dev(pix_subset, torch.int32, "pix_subset")
        if out is None:
            out = torch.empty((npix, L), dtype=torch.float32, device=rgb.device)
        self._dev(out, torch.float32, "loglik")
        prm = params.c()
        subset_ptr = _ptr(pix_subset)
        if pix_subset is not None and pix_subset.numel() == 0:
            # an empty subset is (non-null pointer, count 0); NULL means every pixel
            subset_ptr = ctypes.c_void_p(sample_pix.data_ptr())
        self._sync_stream()
        fn = lib().cs_label_loglik_joint if joint else lib().cs_label_loglik
        self._check(fn(self._h, _ptr(rgb), H, W, _ptr(masks), k,
                       _ptr(sample_pix), _ptr(sample_label), sample_pix.numel(),
                       L, ctypes.byref(prm), subset_ptr,
                       0 if pix_subset is None else pix_subset.numel(),
                       _ptr(out) if out.numel() else None))
        return out

    def label_loglik_soft(self, rgb, alpha, sigma_iota: float, sample_pix, sample_label, L: int,
                          params: Optional[LoglikParams] = None, pix_subset=None,
                          out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """cs_label_loglik_soft: the joint form with smooth co-supports of the
        analysed vectors alpha (N x k float32)."""
        H, W = _image_hw(rgb)
        if alpha.dim() != 2 or alpha.shape[0] != H * W:
            raise ValueError("alpha must be (H*W, k)")
        k = alpha.shape[1]
        _samples(sample_pix, sample_label)
        npix = H * W if pix_subset is None else pix_subset.numel()
        _numel(out, npix * L, "loglik", "npix*L")
        self._dev(rgb, torch.float32, "rgb")
        self._dev(alpha, torch.float32, "alpha")
        self._dev(sample_pix, torch.int32, "sample_pix")
        self._dev(sample_label, torch.int32, "sample_label")
        params = params or LoglikParams()
        if pix_subset is not None:
            self._dev(pix_subset, torch.int32, "pix_subset")
        if out is None:
            out = torch.empty((npix, L), dtype=torch.float32, device=rgb.device)
        self._dev(out, torch.float32, "loglik")
        prm = params.c()
        subset_ptr = _ptr(pix_subset)
        if pix_subset is not None and pix_subset.numel() == 0:
            subset_ptr = ctypes.c_void_p(sample_pix.data_ptr())
        self._sync_stream()
        self._check(lib().cs_label_loglik_soft(self._h, _ptr(rgb), H, W, _ptr(alpha), k,
                                               float(sigma_iota), _ptr(sample_pix),
                                               _ptr(sample_label), sample_pix.numel(), L,
                                               ctypes.byref(prm), subset_ptr,
                                               0 if pix_subset is None else pix_subset.numel(),
                                               _ptr(out) if out.numel() else None))
        return out

    def edge_weight(self, rgb: torch.Tensor, gamma: float = 0.0, out: Optional[torch.Tensor] = None):
        """cs_edge_weight: g (H, W) float32 on the device and the gamma used."""
        H, W = _image_hw(rgb)
        _numel(out, H * W, "g", "H*W")
        self._dev(rgb, torch.float32, "rgb")
        if out is None:
            out = torch.empty((H, W), dtype=torch.float32, device=rgb.device)
        self._dev(out, torch.float32, "g")
        gam = ctypes.c_double()
        self._sync_stream()
        self._check(lib().cs_edge_weight(self._h, _ptr(rgb), H, W, float(gamma), _ptr(out), ctypes.byref(gam)))
        return out, gam.value

    def segment(self, rgb: torch.Tensor, loglik: torch.Tensor, params: "SegmentParams",
                labels: Optional[torch.Tensor] = None, u: Optional[torch.Tensor] = None, want_u: bool = False,
                stats: bool = True):
        """cs_segment: labels (H*W int32), u (H*W, L) float32 or None, and the
        energies (dict, or None without stats)."""
        H, W = _image_hw(rgb)
        if loglik.dim() != 2 or loglik.shape[0] != H * W:
            raise ValueError(f"loglik must be (H*W, L), got {tuple(loglik.shape)}")
        L = int(loglik.shape[1])
        _numel(labels, H * W, "labels", "H*W")
        _numel(u, H * W * L, "u", "H*W*L")
        self._dev(rgb, torch.float32, "rgb")
        self._dev(loglik, torch.float32, "loglik")
        if labels is None:
            labels = torch.empty(H * W, dtype=torch.int32, device=rgb.device)
        self._dev(labels, torch.int32, "labels")
        if u is None and want_u:
            u = torch.empty((H * W, L), dtype=torch.float32, device=rgb.device)
        if u is not None:
            self._dev(u, torch.float32, "u")
        prm = params.c()
        st = _SegmentStatsC()
        self._sync_stream()
        self._check(lib().cs_segment(self._h, _ptr(rgb), H, W, _ptr(loglik), L, ctypes.byref(prm), _ptr(labels),
                                     _ptr(u), ctypes.byref(st) if stats else None))
        info = None
        if stats:
            info = {"primal": st.primal, "binary": st.binary, "dual": st.dual, "gamma": st.gamma,
                    "labels_used": int(st.labels_used)}
        return labels, u, info

    def unsupervised_loglik(self, rgb: torch.Tensor, masks: torch.Tensor, k: int, init_colour, init_texture,
                            params: "UnsupParams", out: Optional[torch.Tensor] = None):
        """cs_unsupervised_loglik: class log-likelihoods (H*W, Kc*Kt) and a dict
        with the colour and texture centroids and classes of every pixel."""
        H, W = _image_hw(rgb)
        _masks_shape(masks, H * W, k)
        Kc, Kt = int(params.colour_classes), int(params.texture_classes)
        ic = (ctypes.c_int32 * max(Kc, 1))(*[int(v) for v in init_colour])
        it = (ctypes.c_int32 * max(Kt, 1))(*[int(v) for v in init_texture])
        if len(init_colour) != Kc or len(init_texture) != Kt:
            raise ValueError("one initial pixel per colour and per texture class")
        _numel(out, H * W * Kc * Kt, "loglik", "H*W*Kc*Kt")
        self._dev(rgb, torch.float32, "rgb")
        self._dev(masks, torch.int64, "masks")
        dev = rgb.device
        if out is None:
            out = torch.empty((H * W, Kc * Kt), dtype=torch.float32, device=dev)
        self._dev(out, torch.float32, "loglik")
        cc = torch.empty((max(Kc, 1), 3), dtype=torch.float64, device=dev)
        tc = torch.empty((max(Kt, 1), _nw(k)), dtype=torch.int64, device=dev)
        cl = torch.empty(H * W, dtype=torch.int32, device=dev)
        tl = torch.empty(H * W, dtype=torch.int32, device=dev)
        prm = params.c()
        self._sync_stream()
        self._check(lib().cs_unsupervised_loglik(self._h, _ptr(rgb), H, W, _ptr(masks), k, ic, it, ctypes.byref(prm),
                                                 _ptr(out), _ptr(cc), _ptr(tc), _ptr(cl), _ptr(tl)))
        return out, {"colour_centroids": cc, "texture_centroids": tc, "colour_labels": cl, "texture_labels": tl}

    def set_check_finite(self, on: bool = True):
        """Optional finite check of rgb and omega before each call (synchronises)."""
        self._check(lib().cs_set_check_finite(self._h, int(bool(on))))

    def last_loglik_stats(self) -> dict:
        st = _LoglikStatsC()
        self._check(lib().cs_last_loglik_stats(self._h, ctypes.byref(st)))
        return {"rescaled_chunks": int(st.rescaled_chunks),
                "overflow_tiles": int(st.overflow_tiles), "exact_tiles": int(st.exact_tiles)}

    def profile_enable(self, on: bool = True):
        self._check(lib().cs_profile_enable(self._h, int(on)))

    def profile_only(self, name: Optional[str]):
        self._check(lib().cs_profile_only(self._h, name.encode() if name else None))

    def profile_sample(self, period: int):
        self._check(lib().cs_profile_sample(self._h, int(period)))

    def profile_read(self, name: str):
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        self._check(lib().cs_profile_read(self._h, name.encode(), ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value


class Mlp:
    """The learned surrogate (one network on the context's device).  The
    initial parameters are an input: a flat float32 tensor (cuda) of
    param_count(in_dim, hidden, out_dim) values."""

    def __init__(self, ctx: Context, in_dim: int, out_dim: int, init_params: torch.Tensor,
                 hidden: int = 128):
        self.ctx = ctx
        self.in_dim, self.hidden, self.out_dim = in_dim, hidden, out_dim
        self.P = param_count(in_dim, hidden, out_dim)
        ctx._dev(init_params, torch.float32, "init_params")
        if self.P and init_params.numel() != self.P:
            raise ValueError(f"init_params must hold {self.P} values")
        self._h = ctypes.c_void_p()
        ctx._sync_stream()
        ctx._check(lib().cs_mlp_init(ctx._h, ctypes.byref(self._h), in_dim, hidden, out_dim,
                                     _ptr(init_params)))

    def close(self):
        if self._h:
            lib().cs_mlp_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _rows(self, x, ell):
        if x.dim() != 2 or x.shape[1] != self.in_dim:
            raise ValueError(f"x must be (n, {self.in_dim}), got {tuple(x.shape)}")
        if ell.dim() != 2 or ell.shape[0] != x.shape[0] or ell.shape[1] != self.out_dim:
            raise ValueError(f"ell must be ({x.shape[0]}, {self.out_dim}), got {tuple(ell.shape)}")

    def params(self) -> torch.Tensor:
        out = torch.empty(self.P, dtype=torch.float32, device=f"cuda:{self.ctx.device}")
        self.ctx._sync_stream()
        self.ctx._check(lib().cs_mlp_get_params(self.ctx._h, self._h, _ptr(out)))
        return out

    def grad(self, x: torch.Tensor, ell: torch.Tensor):
        """(gradient of the mean loss over all rows, loss) without an update."""
        self._rows(x, ell)
        self.ctx._dev(x, torch.float32, "x")
        self.ctx._dev(ell, torch.float32, "ell")
        g = torch.empty(self.P, dtype=torch.float32, device=x.device)
        loss = torch.empty(1, dtype=torch.float32, device=x.device)
        self.ctx._sync_stream()
        self.ctx._check(lib().cs_mlp_grad(self.ctx._h, self._h, _ptr(x), _ptr(ell), x.shape[0],
                                          _ptr(g), _ptr(loss)))
        return g, loss

    def fit_output_bias(self, ell: torch.Tensor):
        """b3 = mean clipped target of each label over the rows of ell."""
        if ell.dim() != 2 or ell.shape[1] != self.out_dim:
            raise ValueError(f"ell must be (n, {self.out_dim})")
        self.ctx._dev(ell, torch.float32, "ell")
        self.ctx._sync_stream()
        self.ctx._check(lib().cs_mlp_fit_output_bias(self.ctx._h, self._h, _ptr(ell), ell.shape[0]))

    def train(self, x: torch.Tensor, ell: torch.Tensor, order: torch.Tensor, batch: int,
              lr: float = 1e-3) -> torch.Tensor:
        """Adam steps over the batches order.view(-1, batch); returns the loss trace."""
        self._rows(x, ell)
        if order.numel() % batch:
            raise ValueError(f"order holds {order.numel()} indices, not a multiple of batch {batch}")
        self.ctx._dev(x, torch.float32, "x")
        self.ctx._dev(ell, torch.float32, "ell")
        self.ctx._dev(order, torch.int32, "order")
        steps = order.numel() // batch
        trace = torch.empty(max(steps, 1), dtype=torch.float32, device=x.device)
        self.ctx._sync_stream()
        self.ctx._check(lib().cs_mlp_train(self.ctx._h, self._h, _ptr(x), _ptr(ell), x.shape[0],
                                           _ptr(order), steps, batch, float(lr), _ptr(trace)))
        return trace[:steps]

    def forward(self, x: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        if x.dim() != 2 or x.shape[1] != self.in_dim:
            raise ValueError(f"x must be (n, {self.in_dim}), got {tuple(x.shape)}")
        n = x.shape[0]
        _numel(out, n * self.out_dim, "out", "n*out_dim")
        self.ctx._dev(x, torch.float32, "x")
        if out is None:
            out = torch.empty((n, self.out_dim), dtype=torch.float32, device=x.device)
        self.ctx._sync_stream()
        self.ctx._check(lib().cs_mlp_forward(self.ctx._h, self._h, _ptr(x), n, _ptr(out)))
        return out

    def infer(self, rgb: torch.Tensor, alpha: torch.Tensor, out: Optional[torch.Tensor] = None):
        H, W = _image_hw(rgb)
        k = self.in_dim - 5
        _numel(alpha, H * W * k, "alpha", "H*W*(in_dim-5)")
        _numel(out, H * W * self.out_dim, "out", "H*W*out_dim")
        self.ctx._dev(rgb, torch.float32, "rgb")
        self.ctx._dev(alpha, torch.float32, "alpha")
        if out is None:
            out = torch.empty((H * W, self.out_dim), dtype=torch.float32, device=rgb.device)
        self.ctx._sync_stream()
        self.ctx._check(lib().cs_mlp_infer(self.ctx._h, self._h, _ptr(rgb), H, W, _ptr(alpha), k,
                                           _ptr(out)))
        return out


    def infer_fallback(self, rgb: torch.Tensor, alpha: torch.Tensor, masks: torch.Tensor, kmask: int,
                       sample_pix: torch.Tensor, sample_label: torch.Tensor, params: Optional[LoglikParams] = None,
                       margin: float = 2.0, out: Optional[torch.Tensor] = None):
        """Inference with the exact data term for the pixels whose two largest
        outputs differ by less than `margin` nats; returns (out, pixels
        recomputed exactly)."""
        H, W = _image_hw(rgb)
        k = self.in_dim - 5
        _numel(alpha, H * W * k, "alpha", "H*W*(in_dim-5)")
        _numel(out, H * W * self.out_dim, "out", "H*W*out_dim")
        _masks_shape(masks, H * W, kmask)
        _samples(sample_pix, sample_label)
        for t, dt, nm in ((rgb, torch.float32, "rgb"), (alpha, torch.float32, "alpha"), (masks, torch.int64, "masks"),
                          (sample_pix, torch.int32, "sample_pix"), (sample_label, torch.int32, "sample_label")):
            self.ctx._dev(t, dt, nm)
        if out is None:
            out = torch.empty((H * W, self.out_dim), dtype=torch.float32, device=rgb.device)
        prm = (params or LoglikParams()).c()
        n = ctypes.c_int64()
        self.ctx._sync_stream()
        self.ctx._check(lib().cs_mlp_infer_fallback(self.ctx._h, self._h, _ptr(rgb), H, W, _ptr(alpha), k, _ptr(masks),
                                                    kmask, _ptr(sample_pix), _ptr(sample_label), sample_pix.numel(),
                                                    self.out_dim, ctypes.byref(prm), float(margin), _ptr(out),
                                                    ctypes.byref(n)))
        return out, int(n.value)


def param_count(in_dim: int, hidden: int, out_dim: int) -> int:
    return int(lib().cs_mlp_param_count(in_dim, hidden, out_dim))


def mlp_features(ctx: Context, rgb: torch.Tensor, alpha: torch.Tensor, pix: torch.Tensor,
                 out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Surrogate input rows of the pixels `pix` (int32, cuda)."""
    H, W = _image_hw(rgb)
    if alpha.dim() != 2 or alpha.shape[0] != H * W:
        raise ValueError("alpha must be (H*W, k)")
    k = alpha.shape[1]
    _numel(out, pix.numel() * (5 + k), "out", "n*(5+k)")
    ctx._dev(rgb, torch.float32, "rgb")
    ctx._dev(alpha, torch.float32, "alpha")
    ctx._dev(pix, torch.int32, "pix")
    if out is None:
        out = torch.empty((pix.numel(), 5 + k), dtype=torch.float32, device=rgb.device)
    ctx._sync_stream()
    ctx._check(lib().cs_mlp_features(ctx._h, _ptr(rgb), H, W, _ptr(alpha), k, _ptr(pix),
                                     pix.numel(), _ptr(out)))
    return out
