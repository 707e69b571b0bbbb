"""MI355X-native co-sparse data term (arXiv 1312.4746) -- Python binding.

A thin ctypes layer over the C-ABI of ``libcosparse.so`` (declared in
``include/cosparse.h``): it checks tensor shapes, dtypes and devices and
passes raw device pointers and torch's current HIP stream.  Every step of the
computation runs in the library's HIP kernels; there is no fallback path, and
loading fails loudly when the library has not been built.
"""
from __future__ import annotations

from .binding import (  # noqa: F401
    CS_BF16,
    CS_FP32,
    Context,
    CosparseError,
    LoglikParams,
    Mlp,
    SegmentParams,
    UnsupParams,
    lib,
    library_path,
    mlp_features,
    param_count,
)
