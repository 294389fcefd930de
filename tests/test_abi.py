"""The C-ABI library loads and exports every entry point include/amm.h declares
(no GPU work), and the binding's declarations match the header."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "amm.h")
LIB = os.path.join(ROOT, "paper_2504_19308_amd", "libamm.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(amm_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("amm_decompose", "amm_approx_matmul", "amm_dec_import_circulant",
                     "amm_dec_import_tsvd", "amm_dec_import_sparse", "amm_ctx_create"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libamm.so not built")
def test_library_exports_every_declared_symbol():
    import ctypes
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libamm.so not built")
def test_binding_covers_header():
    from paper_2504_19308_amd import _lib
    assert set(_lib.SIGNATURES) == set(declared_functions())
    lib = _lib.load()
    o = _lib.AmmOpts()
    lib.amm_opts_default(o)
    assert o.oversample == 16 and o.power_iters == 2 and o.keep_residual == 1
    assert abs(o.sparse_frac - 0.01) < 1e-15 and o.sparse_nnz == -1


@pytest.mark.skipif(not os.path.exists(LIB), reason="libamm.so not built")
def test_null_arguments_are_rejected_without_a_device():
    import ctypes
    from paper_2504_19308_amd import _lib
    lib = _lib.load()
    assert lib.amm_approx_matmul(None, None, None, None, 4, 4, None, None) == 1  # AMM_EINVAL
    assert lib.amm_last_error().decode() != ""
    assert lib.amm_dec_query(None, None) == 1
    assert lib.amm_ctx_create(None, 0) == 1
