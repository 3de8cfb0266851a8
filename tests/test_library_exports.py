"""CPU-side checks of the C ABI library: it loads and exports every symbol
include/ufvc.h declares (no compute calls: there may be no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ufvc.h")
LIB = os.path.join(ROOT, "paper_2606_04410_amd", "libufvc.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ufvc_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ("ufvc_create", "ufvc_destroy", "ufvc_encode_chunk", "ufvc_decode_chunk",
                 "ufvc_rans_encode", "ufvc_rans_decode", "ufvc_get_tables"):
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libufvc.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing
    import paper_2606_04410_amd as pkg
    assert sorted(pkg.EXPORTS) == declared()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libufvc.so not built")
def test_weight_count_matches_generator():
    import paper_2606_04410_amd as pkg
    from synthetic import weight_shapes
    import numpy as np
    for T, C in ((4, 64), (8, 128), (1, 128)):
        n = sum(int(np.prod(s)) for _, s in weight_shapes(T, C))
        assert pkg.lib.ufvc_weight_count(T, C) == n
    assert pkg.lib.ufvc_weight_count(9, 128) == 0
