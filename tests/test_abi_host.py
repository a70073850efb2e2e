"""The C ABI on the CPU: the library loads, exports every function that
include/bkwd.h declares, and rejects bad arguments before any device work."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bkwd.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bkwd_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def B():
    from paper_0903_4936_amd import bkwd
    if not os.path.exists(bkwd.LIB_PATH):
        from paper_0903_4936_amd import build
        build.build()
    return bkwd


def test_every_declared_symbol_is_exported(B):
    lib = B.lib()
    names = _declared()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
        assert n in B.SIGNATURES, n


def test_lattice_bytes(B):
    n = B.lattice_bytes((4, 4, 4, 4))
    V = 256
    # links FP64 + FP32 + copy, clover FP64 + FP32
    assert n >= V * (36 * 16 + 36 * 8 + 36 * 16 + 72 * 8 + 72 * 4)
    assert B.lattice_bytes((4, 4, 4, 4), B.COMPRESS12) > n
    assert B.lattice_bytes((4, 1, 4, 4)) == 0


def test_create_rejects_bad_arguments(B):
    lib = B.lib()
    h = ctypes.c_void_p(1)
    dims = (ctypes.c_int * 4)(4, 4, 4, 4)
    links = (ctypes.c_double * 8)()
    assert lib.bkwd_lattice_create(dims, None, 0.1, 1.0, 0, ctypes.c_void_p(256), 1 << 30, None,
                                   ctypes.byref(h)) == B.EINVAL
    assert h.value is None
    assert "links" in B.last_error()
    bad = (ctypes.c_int * 4)(4, 1, 4, 4)
    assert lib.bkwd_lattice_create(bad, links, 0.1, 1.0, 0, ctypes.c_void_p(256), 1 << 30, None,
                                   ctypes.byref(h)) == B.EINVAL
    assert "extent" in B.last_error()
    assert lib.bkwd_lattice_create(dims, links, 0.1, 1.0, 0, ctypes.c_void_p(8), 1 << 30, None,
                                   ctypes.byref(h)) == B.EINVAL
    assert "aligned" in B.last_error()
    assert lib.bkwd_lattice_create(dims, links, 0.1, 1.0, 0, ctypes.c_void_p(256), 16, None,
                                   ctypes.byref(h)) == B.ENOMEM
    assert lib.bkwd_lattice_create(dims, links, float("nan"), 1.0, 0, ctypes.c_void_p(256), 1 << 30, None,
                                   ctypes.byref(h)) == B.EINVAL


def test_null_handle_calls(B):
    lib = B.lib()
    assert lib.bkwd_apply(None, 0, 12, B.FP64, ctypes.c_void_p(256), ctypes.c_void_p(512), None) == B.EINVAL
    o = B.default_opts()
    info = B.SolveInfo()
    assert lib.bkwd_block_solve(None, 12, None, None, ctypes.byref(o), None, 0, ctypes.byref(info),
                                None) == B.EINVAL
    assert lib.bkwd_solve_workspace_bytes(None, 12, ctypes.byref(o)) == 0
    assert lib.bkwd_lattice_destroy(None) == B.OK
    assert lib.bkwd_lattice_set_params(None, 0.1, 1.0, None) == B.EINVAL


def test_default_opts(B):
    o = B.default_opts()
    assert o.method == B.BLOCK_BICGGR and o.prec == B.MIXED
    assert o.tol == 1e-12 and o.inner_tol == 0.0  # 0: chosen by L at solve time
    assert o.qr_frame == -1  # -1: chosen by precision at solve time
    assert o.max_block == 0  # 0: chosen by precision and L at solve time
    assert o.max_iter > 0 and o.check_every >= 1
