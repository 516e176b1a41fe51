"""CPU checks of the BLAS offload layer (liboz_blas.so): it loads, exports
what include/oz_blas.h declares, parses modes, and reports illegal arguments
with the reference BLAS parameter numbers without starting any GPU work;
quick returns leave C alone without touching the device."""
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "oz_blas.h")


def declared():
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:void|int)\s+(\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def blas():
    import paper_2503_22875_amd.blas as b
    return b


def test_exports_every_declared_symbol(blas):
    names = declared()
    assert names == sorted(blas.EXPORTS)
    for n in names:
        assert hasattr(blas._lib, n)


def test_mode_strings(blas):
    assert blas.oz_blas_set_mode("fp64_int8_3") and blas.oz_blas_stats().slices == 3
    assert blas.oz_blas_set_mode("fp64_int8_18") and blas.oz_blas_stats().slices == 18
    assert blas.oz_blas_set_mode("fp64_int8_tol1e-10")
    st = blas.oz_blas_stats()
    assert st.mode == 2 and st.tol == 1e-10
    assert blas.oz_blas_set_mode("dgemm") and blas.oz_blas_stats().mode == 0
    assert blas.oz_blas_set_mode("fp64_int8_bal6")
    st = blas.oz_blas_stats()
    assert st.mode == 3 and st.slices == 6
    for bad in ("fp64_int8_0", "fp64_int8_19", "fp64_int8_", "fp64_int8_tol", "fp64_int8_tol-1", "int8", "",
                "fp64_int8_7x", "fp64_int8_bal", "fp64_int8_bal0", "fp64_int8_bal9", "fp64_int8_bal6x"):
        assert not blas.oz_blas_set_mode(bad), bad
    assert blas.oz_blas_set_mode("fp64_int8_7") and blas.oz_blas_stats().mode == 1


@pytest.mark.parametrize("field,value,info", [
    ("ta", "X", 1), ("tb", "Q", 2), ("m", -1, 3), ("n", -2, 4), ("k", -3, 5),
    ("lda", 3, 8), ("ldb", 4, 10), ("ldc", 3, 13),
])
def test_illegal_arguments(blas, field, value, info):
    a = dict(ta="N", tb="N", m=4, n=5, k=6, lda=4, ldb=6, ldc=4)
    a[field] = value
    A = np.zeros((4, 6), order="F")
    B = np.zeros((6, 5), order="F")
    C = np.full((4, 5), 3.0, order="F")
    calls = blas.oz_blas_stats().calls
    blas.dgemm_(a["ta"], a["tb"], a["m"], a["n"], a["k"], 1.0, A, a["lda"], B, a["ldb"], 0.0, C, a["ldc"])
    st = blas.oz_blas_stats()
    assert st.last_info == info and st.calls == calls
    assert np.all(C == 3.0)
    Z = np.zeros((4, 5), np.complex128, order="F")
    blas.zgemm_(a["ta"], a["tb"], a["m"], a["n"], a["k"], 1.0, A, a["lda"], B, a["ldb"], 0.0, Z, a["ldc"])
    assert blas.oz_blas_stats().last_info == info


def test_lowercase_trans_and_quick_returns(blas):
    A = np.ones((3, 3), order="F")
    C = np.full((3, 3), 2.0, order="F")
    calls = blas.oz_blas_stats().calls
    blas.dgemm_("n", "t", 0, 3, 3, 1.0, A, 3, A, 3, 0.0, C, 3)       # m = 0
    blas.dgemm_("n", "t", 3, 3, 3, 0.0, A, 3, A, 3, 1.0, C, 3)       # alpha = 0, beta = 1
    blas.dgemm_("c", "c", 3, 3, 0, 1.0, A, 3, A, 3, 1.0, C, 3)       # k = 0, beta = 1
    st = blas.oz_blas_stats()
    assert st.last_info == 0 and st.calls == calls
    assert np.all(C == 2.0)
