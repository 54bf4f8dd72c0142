"""CPU checks of the C ABI: the built library loads and exports every function
that include/mvgeo.h declares (no compute calls: there is no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mvgeo.h")
SO = os.path.join(ROOT, "paper_2008_07437_amd", "libmvgeo.so")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = set()
    for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b([A-Za-z_]\w*)\s*\(", src, re.M):
        name = m.group(1)
        if name not in ("if", "while", "for", "sizeof", "defined"):
            names.add(name)
    return names


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("cov_generate", "potrf_tiled", "loglik", "tlr_compress", "cokrige_predict",
              "morton_order", "mvg_footprint", "mvg_last_error"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(SO), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(SO)
    for name in sorted(_declared()):
        assert hasattr(lib, name), name
    lib.mvg_last_error.restype = ctypes.c_char_p
    assert lib.mvg_last_error() == b""


def test_product_path_fails_without_gpu_or_library(monkeypatch):
    import torch
    import paper_2008_07437_amd._lib as L
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    monkeypatch.setattr(L, "_lib", None)
    with pytest.raises((ImportError, RuntimeError)):
        L._load()
