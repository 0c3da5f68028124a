"""The C-ABI library loads and exports every entry point declared in include/fiohss.h (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fiohss.h")
LIB = os.path.join(ROOT, "paper_2609_11520_amd", "libfiohss.so")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_ ]*?[\s\*]+([a-z_][a-z0-9_]*)\s*\(", txt, flags=re.M)
    return sorted(set(n for n in names if n.startswith(("fio_", "hss_"))))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("fio_bf_apply", "fio_bf_apply_adj", "hss_build_from_samples", "hss_ulv_factor", "hss_ulv_solve",
              "fio_approx_solve", "fio_bf_build", "fio_bf_import"):
        assert n in names, n


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_prototypes_match_header():
    from paper_2609_11520_amd import _lib
    assert sorted(_lib.PROTOS) == declared_functions()


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_host_side_argument_checks_without_gpu():
    # calls that fail argument validation return before touching the device
    from paper_2609_11520_amd import _lib
    lib = _lib.load()
    d = _lib.BfDesc(1, 1000, 0.0, 0.0, 9, 3, 1)          # N not a power of two
    assert lib.fio_bf_factor_count(ctypes.byref(d)) == 0
    d = _lib.BfDesc(1, 1 << 10, 0.125, 0.0625, 9, 3, 1)
    # V + 2 (L'-h) transfer factors + M + U  =  N (2*8q + q^2 + 2 (L'-h) 2 q^2)
    assert lib.fio_bf_factor_count(ctypes.byref(d)) == (1 << 10) * (2 * 8 * 9 + 81 + 2 * 2 * 2 * 81)
    d = _lib.BfDesc(1, 1 << 11, 0.125, 0.0625, 9, 3, 1)  # odd L is not implemented
    h = ctypes.c_void_p()
    assert lib.fio_bf_build(ctypes.byref(d), None, ctypes.byref(h)) == -6
    assert lib.fio_bf_apply(None, None, 0, None, 0, 1, 0, None, 0, None) == -1
    assert lib.fio_status_str(-4) == b"matrix not Hermitian positive definite"
    r = (ctypes.c_int * 2)(3, 4)
    # one level: U of two leaves (8 x r) + B (r2 x r1) + two 8 x 8 leaves
    assert lib.hss_generator_count(16, 8, r) == 8 * 3 + 8 * 4 + 4 * 3 + 2 * 64
