"""The C-ABI library loads on the host and exports every entry point that
include/cosparse.h declares; the Python binding covers the same set.  No
compute call is made (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cosparse.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cs_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def so_path():
    from paper_1312_4746_amd import build as b
    if not os.path.exists(b.SO):
        b.build()
    return b.SO


def test_header_declares_the_four_paper_calls():
    names = _declared()
    for n in ("cs_analyze_patches", "cs_cosupport", "cs_texture_similarity", "cs_label_loglik"):
        assert n in names


def test_library_exports_every_declared_symbol(so_path):
    lib = ctypes.CDLL(so_path)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_signatures_cover_header(so_path):
    from paper_1312_4746_amd.binding import SIGNATURES
    assert sorted(SIGNATURES) == _declared()


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    import paper_1312_4746_amd.binding as bnd
    monkeypatch.setattr(bnd, "_lib", None)
    monkeypatch.setattr(bnd, "_SO", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError):
        bnd.lib()


def test_oracle_and_library_share_no_source():
    """The oracle is independent of the HIP path: no include or import crosses over."""
    lib_dir = os.path.join(ROOT, "paper_1312_4746_amd")
    for dp, _, files in os.walk(lib_dir):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dp, f)).read()
                assert "cso_" not in txt and "import oracle" not in txt and "from oracle" not in txt
    for f in os.listdir(os.path.join(ROOT, "oracle")):
        if f.endswith((".c", ".h", ".py")):
            txt = open(os.path.join(ROOT, "oracle", f)).read()
            assert "cosparse.h" not in txt and "paper_1312_4746_amd" not in txt
