"""The binding checks buffer shapes before any launch: the C layer sees only
device pointers and sizes, so a buffer of the wrong size would be read or
written out of bounds on the GPU.  Each check raises ValueError from tensor
metadata alone, before the device or dtype checks and before any library
call, so these tests run on the CPU with host tensors."""
import ctypes
import os
import re

import pytest
import torch

from paper_1312_4746_amd import binding as bnd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


class _NoLib:
    def __getattr__(self, name):
        raise AssertionError(f"library call {name} reached before the shape check")


@pytest.fixture
def ctx(monkeypatch):
    monkeypatch.setattr(bnd, "_lib", _NoLib())
    c = bnd.Context.__new__(bnd.Context)
    c.device = 0
    c._h = ctypes.c_void_p()
    return c


def f32(*s):
    return torch.zeros(s, dtype=torch.float32)


def i32(*s):
    return torch.zeros(s, dtype=torch.int32)


def i64(*s):
    return torch.zeros(s, dtype=torch.int64)


def test_rgb_must_be_three_planes(ctx):
    with pytest.raises(ValueError, match="rgb"):
        ctx.analyze_patches(f32(4, 8, 8), 3, 1.0, f32(5, 9))
    with pytest.raises(ValueError, match="rgb"):
        ctx.analyze_patches(f32(8, 8), 3, 1.0, f32(5, 9))


def test_omega_must_match_patch_size(ctx):
    with pytest.raises(ValueError, match="omega"):
        ctx.analyze_patches(f32(3, 8, 8), 3, 1.0, f32(5, 10))


def test_alpha_out_size(ctx):
    with pytest.raises(ValueError, match="alpha"):
        ctx.analyze_patches(f32(3, 8, 8), 3, 1.0, f32(5, 9), out=f32(64, 4))
    with pytest.raises(ValueError, match="alpha"):
        ctx.tau_median(f32(3, 8, 8), 3, 1.0, f32(5, 9), f32(63, 5))
    with pytest.raises(ValueError, match="alpha"):
        ctx.cosupport(f32(3, 8, 8), 3, 1.0, f32(5, 9), 0.1, alpha=f32(64, 6))
    with pytest.raises(ValueError, match="alpha"):
        ctx.cosupport_median(f32(3, 8, 8), 3, 1.0, f32(5, 9), alpha=f32(10))


def test_masks_shape(ctx):
    # k = 65 needs two words per pixel
    with pytest.raises(ValueError, match="masks"):
        ctx.cosupport(f32(3, 8, 8), 3, 1.0, f32(65, 9), 0.1, out=i64(64, 1))
    with pytest.raises(ValueError, match="masks"):
        ctx.cosupport_median(f32(3, 8, 8), 3, 1.0, f32(65, 9), out=i64(64, 1))
    with pytest.raises(ValueError, match="masks"):
        ctx.label_loglik(f32(3, 8, 8), i64(64, 1), 65, i32(4), i32(4), 2)
    with pytest.raises(ValueError, match="masks"):
        ctx.label_loglik(f32(3, 8, 8), i64(63, 1), 10, i32(4), i32(4), 2)
    with pytest.raises(ValueError, match="A"):
        ctx.texture_similarity(i64(5, 1), i64(5, 2), 100)
    with pytest.raises(ValueError, match="B"):
        ctx.texture_similarity(i64(5, 2), i64(5), 100)


def test_sample_lists_agree(ctx):
    with pytest.raises(ValueError, match="sample_label"):
        ctx.label_loglik(f32(3, 8, 8), i64(64, 1), 10, i32(4), i32(5), 2)
    with pytest.raises(ValueError, match="sample_label"):
        ctx.label_loglik_soft(f32(3, 8, 8), f32(64, 10), 0.01, i32(4), i32(3), 2)


def test_loglik_out_size(ctx):
    with pytest.raises(ValueError, match="loglik"):
        ctx.label_loglik(f32(3, 8, 8), i64(64, 1), 10, i32(4), i32(4), 2, out=f32(64, 3))
    with pytest.raises(ValueError, match="loglik"):
        ctx.label_loglik(f32(3, 8, 8), i64(64, 1), 10, i32(4), i32(4), 2, pix_subset=i32(7), out=f32(64, 2))
    with pytest.raises(ValueError, match="loglik"):
        ctx.label_loglik_soft(f32(3, 8, 8), f32(64, 10), 0.01, i32(4), i32(4), 2, out=f32(10))
    with pytest.raises(ValueError, match="alpha"):
        ctx.label_loglik_soft(f32(3, 8, 8), f32(63, 10), 0.01, i32(4), i32(4), 2)


def test_tsm_out_size(ctx):
    with pytest.raises(ValueError, match="out"):
        ctx.texture_similarity(i64(5, 1), i64(6, 1), 10, out=i32(5, 5))


def test_mlp_shapes(ctx):
    net = bnd.Mlp.__new__(bnd.Mlp)
    net.ctx, net.in_dim, net.hidden, net.out_dim, net.P = ctx, 103, 128, 10, 31114
    net._h = ctypes.c_void_p()
    with pytest.raises(ValueError, match="x"):
        net.grad(f32(16, 102), f32(16, 10))
    with pytest.raises(ValueError, match="ell"):
        net.grad(f32(16, 103), f32(15, 10))
    with pytest.raises(ValueError, match="order"):
        net.train(f32(32, 103), f32(32, 10), i32(40), 16)
    with pytest.raises(ValueError, match="x"):
        net.forward(f32(16, 100))
    with pytest.raises(ValueError, match="out"):
        net.forward(f32(16, 103), out=f32(16, 9))
    with pytest.raises(ValueError, match="alpha"):
        net.infer(f32(3, 8, 8), f32(64, 97))
    with pytest.raises(ValueError, match="out"):
        net.infer(f32(3, 8, 8), f32(64, 98), out=f32(64, 11))
    with pytest.raises(ValueError, match="ell"):
        net.fit_output_bias(f32(16, 9))
    with pytest.raises(ValueError, match="out"):
        bnd.mlp_features(ctx, f32(3, 8, 8), f32(64, 10), i32(5), out=f32(5, 14))


def test_nonfinite_status_is_declared_and_mapped():
    src = open(os.path.join(ROOT, "include", "cosparse.h")).read()
    m = re.search(r"#define\s+CS_ERR_NONFINITE\s+(\d+)", src)
    assert m and int(m.group(1)) == bnd.CS_ERR_NONFINITE == 5
    e = bnd.CosparseError(bnd.CS_ERR_NONFINITE, "an input holds a NaN")
    assert e.code == 5 and "NaN" in str(e)
