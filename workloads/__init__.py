"""Seeded synthetic workloads for the co-sparse data term.

This package only draws inputs (images, analysis operators, scribble
samples, training-pixel subsets, initial surrogate weights and data order,
the pixels that start the unsupervised clustering).  It contains none of the method's
arithmetic, so both the FP64 oracle and the HIP library can be fed from
it without sharing any computation.
"""
from .gen import (  # noqa: F401
    CONFIGS,
    Workload,
    make_config,
    make_workload,
    make_omega,
    mlp_init,
    mlp_order,
    quantise_colours,
    unsup_init,
)
