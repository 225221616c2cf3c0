"""The C-ABI library loads and exports every entry point include/qpat.h declares
(host-only checks: no device work is launched here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qpat.h")
LIB = os.path.join(ROOT, "paper_1512_02796_amd", "libqpat.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qpat_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_path():
    names = declared_functions()
    for want in ("qpat_setup_mesh", "qpat_forward", "qpat_jvp", "qpat_vjp", "qpat_prior_apply",
                 "qpat_prior_solve", "qpat_prior_setup", "qpat_lsqr_init", "qpat_lsqr_step",
                 "qpat_destroy", "qpat_last_error"):
        assert want in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libqpat.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libqpat.so not built")
def test_binding_signatures_cover_header_and_defaults():
    from paper_1512_02796_amd import qpat
    assert set(qpat.SIGNATURES) == set(declared_functions())
    o = qpat.default_opts()        # host-only entry point
    assert o.precision == 0 and o.max_rhs_block == 16 and o.pcg_rtol == 1e-10
    assert o.prior_deflate == 1 and o.lsqr_reorth == 1
    assert "gfx950" in qpat.version()
