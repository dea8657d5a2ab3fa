"""CPU checks of the C ABI: the library loads, exports every function that
include/dlma.h declares, and rejects bad arguments before touching the GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dlma.h")
LIB = os.path.join(ROOT, "paper_2201_09729_amd", "libdlma.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dlma_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2201_09729_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("dlma_load_gauge", "dlma_apply_dw", "dlma_solve", "dlma_lap_eigs", "dlma_project", "dlma_correlators"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_argument_validation_without_gpu(lib):
    lib.dlma_last_error.restype = ctypes.c_char_p
    lib.dlma_version.restype = ctypes.c_char_p
    assert b"gfx950" in lib.dlma_version()
    h = ctypes.c_void_p()
    U = ctypes.c_void_p(1)  # never dereferenced: validation fails first
    for dims in ((4, 4, 4, 3), (0, 4, 4, 4), (4, 4, 4, 8192), (512, 512, 512, 2)):
        d = (ctypes.c_int * 4)(*dims)
        rc = lib.dlma_load_gauge(d, U, ctypes.c_double(0.12), ctypes.c_double(1.0), None, ctypes.byref(h))
        assert rc == -1, dims
        assert len(lib.dlma_last_error()) > 0
    d = (ctypes.c_int * 4)(4, 4, 4, 4)
    assert lib.dlma_load_gauge(d, U, ctypes.c_double(-0.1), ctypes.c_double(1.0), None, ctypes.byref(h)) == -1
    assert lib.dlma_load_gauge(d, U, ctypes.c_double(0.12), ctypes.c_double(-1.0), None, ctypes.byref(h)) == -1
    assert lib.dlma_load_gauge(d, None, ctypes.c_double(0.12), ctypes.c_double(1.0), None, ctypes.byref(h)) == -1
    assert lib.dlma_solve(None, 1, None, None, None, None) == -1
    assert lib.dlma_apply_dw(None, None, None, 1, 0, None) == -1
    assert lib.dlma_apply_schur(None, None, None, 1, 0, 2, 0, 0, 1, None) == -1
    assert lib.dlma_lap_eigs(None, 4, 0, 1, None, None, None, None, None) == -1
    assert lib.dlma_project(None, 0, 1, None, None, None, 1, 0, None) == -1
    assert lib.dlma_correlators(None, 0, 1, None, None, 1, 0, 1, None, None, None, None) == -1
    assert lib.dlma_correlators_grad(None, 0, 1, None, None, 1, 0, 1, None, None, None, None, None, None, None) == -1
    assert lib.dlma_project_noalloc(None, 0, 1, None, None, None, 1, 0, None) == -1
    assert lib.dlma_profile_read(10, None, None, None) == -1  # classes are 0..9
    assert lib.dlma_release_cache() == 0  # nothing cached: no device call


def test_solve_opts_defaults(lib):
    from paper_2201_09729_amd.dlma import SolveOpts
    o = SolveOpts()
    lib.dlma_solve_opts_default(ctypes.byref(o))
    assert o.tol == 1e-10 and o.prec == 0 and o.rhs_block == 0 and o.max_outer > 0
