"""CPU checks of the boundary: the library loads, exports every symbol that
include/chfsi.h declares, and rejects invalid arguments before touching a GPU."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "chfsi.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(chfsi_[a-zA-Z_0-9]+)\s*\(", src)))


def test_library_exports_header_symbols():
    import paper_2410_02754_amd as pkg
    lib = pkg.load()
    names = _declared()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(pkg._lib.EXPORTED)
    assert lib.chfsi_version().startswith(b"chfsi")


def test_create_rejects_bad_arguments():
    import paper_2410_02754_amd._lib as L
    lib = L.load()
    k = (C.c_double * 3)(0, 0, 0)
    for nc, p, nq in [((1, 2, 2), 3, 4), ((2, 2, 2), 0, 4), ((2, 2, 2), 9, 4), ((2, 2, 2), 3, 0)]:
        d = L.MeshDesc()
        d.n_cells = (C.c_int * 3)(*nc)
        d.box = (C.c_double * 3)(4, 4, 4)
        d.p, d.quad, d.n_q, d.n_k = p, 0, nq, 1
        d.kpts = C.cast(k, C.POINTER(C.c_double))
        ctx = C.c_void_p()
        assert lib.chfsi_create(C.byref(d), None, C.byref(ctx)) == -1
        assert lib.chfsi_last_error(None)
    assert lib.chfsi_create(None, None, None) == -1
    assert lib.chfsi_destroy(None) == 0
    assert lib.chfsi_apply_H(None, 0, None, 1, None, 1, 1, 0) == -1


def test_no_oracle_in_product_path():
    """The package never imports the oracle or a CPU fallback."""
    pkg = os.path.join(ROOT, "paper_2410_02754_amd")
    for f in os.listdir(pkg):
        if f.endswith(".py"):
            text = open(os.path.join(pkg, f)).read()
            assert "oracle" not in re.sub(r'""".*?"""', "", text, flags=re.S), f
