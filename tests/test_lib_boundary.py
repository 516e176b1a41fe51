"""CPU checks of the C-ABI library: it loads, it exports every function that
include/oz.h declares, and its host-only paths (layout sizes, status text,
handle and argument checks) behave as documented.  No GPU work is started."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "oz.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\**\s+\**(oz_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ["oz_create", "oz_destroy", "oz_dgemm", "oz_zgemm", "oz_split", "oz_diag_sums"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_2503_22875_amd as oz
    lib = ctypes.CDLL(oz.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert sorted(oz.EXPORTS) == declared_functions()


def test_status_strings():
    import paper_2503_22875_amd as oz
    assert oz.oz_status_string(0) == "success"
    assert "Inf" in oz.oz_status_string(oz.OZ_ERR_NONFINITE)
    assert "position" in oz.oz_status_string(8)


@pytest.mark.parametrize("side,cplx,nv,k,s,rows,kpad", [
    ("A", 0, 256, 256, 7, 256, 256),
    ("A", 0, 1, 1, 1, 128, 32),
    ("B", 0, 65, 33, 3, 128, 64),
    ("A", 1, 100, 37, 7, 256, 96),   # 2*ceil(100/16)*16 = 224 rows -> 256; 74 terms -> 96
    ("B", 1, 100, 37, 7, 128, 96),
    ("A", 1, 4096, 4096, 7, 8192, 8192),
])
def test_split_layout_sizes(side, cplx, nv, k, s, rows, kpad):
    import paper_2503_22875_amd as oz
    rp, kp, nb = oz.oz_split_layout(side, cplx, nv, k, s)
    assert (rp, kp, nb) == (rows, kpad, s * rows * kpad)


def test_invalid_handle_and_arguments_are_rejected_on_host():
    import paper_2503_22875_amd as oz
    st = oz.oz_dgemm(None, "N", "N", 4, 4, 4, 1.0, None, 4, None, 4, 0.0, None, 4, check=False)
    assert st == oz.OZ_ERR_HANDLE
    with pytest.raises(oz.OzError):
        oz.oz_split_layout("X", 0, 4, 4, 7)
    with pytest.raises(oz.OzError):
        oz.oz_split_layout("A", 0, 4, 4, 19)


def test_product_path_has_no_oracle_or_cpu_fallback():
    pkg = os.path.join(ROOT, "paper_2503_22875_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "oz_oracle" not in text, f
