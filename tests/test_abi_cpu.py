"""Host-side checks of the C ABI library that need no GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2512_22215_amd", "libldu.so")
HDR = os.path.join(ROOT, "include", "ldu.h")
BENCH_HDR = os.path.join(ROOT, "include", "ldu_bench.h")


def _declared(hdr=HDR):
    src = open(hdr).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b([a-z_][a-z0-9_]*)\s*\(", src)) - {"if", "sizeof"})


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("ldu_create", "ldu_amul", "ldu_tmul", "pcg_solve", "gamg_solve",
                     "ldu_adjoint_solve", "ldu_coeff_grad", "ldu_set_coeffs"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libldu.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in _declared():
        assert hasattr(lib, name), name
    from paper_2512_22215_amd import ldu
    assert sorted(ldu.EXPORTED) == sorted(_declared())
    for name in _declared(BENCH_HDR):
        assert hasattr(lib, name), name
    assert sorted(ldu.BENCH_EXPORTED) == sorted(_declared(BENCH_HDR))


@pytest.mark.skipif(not os.path.exists(LIB), reason="libldu.so not built")
def test_default_options_and_null_arguments():
    from paper_2512_22215_amd import ldu
    o = ldu.pcg_opts()
    assert o.rel_tol == 1e-8 and o.max_iter == 10000 and o.precond == 1
    g = ldu.gamg_opts()
    assert g.omega == 0.75 and g.n_pre == 2 and g.n_post == 2 and g.n_coarsest == 50
    assert g.passes == 1
    h = ctypes.c_void_p()
    # argument checks happen before any device call
    assert ldu.lib().ldu_create(0, 0, None, None, None, None, None, None,
                                ctypes.byref(h)) == ldu.LDU_ERR_ARG
    assert ldu.lib().ldu_amul(None, None, None, None) == ldu.LDU_ERR_ARG
    assert b"NULL" in ldu.lib().ldu_last_error()
