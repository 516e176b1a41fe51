"""The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

The oracle allocates with malloc and indexes digit planes, chunks and strided
operands by hand.  This test builds the same source with -fsanitize=address,
undefined (every report fatal), runs a spread of oracle calls in a child
process that preloads the ASan runtime -- ragged and empty sizes, every trans,
strided views of padded buffers, forced INT32 chunks, incremental
growth, balanced digits, the 3-product form, double-double results, row and
column subsets, Inf/NaN and subnormal inputs -- and checks that the child
exits cleanly with no sanitizer report and that every result equals, bit for
bit, the same call on the regular build.
"""
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
from oracle import build as obuild

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# The cases, run once in the sanitized child and once here on the regular build.
CASES_SRC = r'''
import numpy as np
import oracle

rng = np.random.default_rng(11)

def mat(r, c, cplx=False, ld=None):
    X = rng.standard_normal((r, c)) * np.ldexp(1.0, rng.integers(-30, 31, size=(r, 1)))
    if cplx:
        X = X + 1j * rng.standard_normal((r, c))
    ld = r if ld is None else ld
    buf = np.zeros((max(ld, 1), c), dtype=X.dtype, order="F")
    buf[:r] = X
    return buf[:r], X

def op_shape(trans, rows, cols):
    return (rows, cols) if trans == "N" else (cols, rows)

def cases():
    out = {}
    for cplx in (False, True):
        tr = "NTC" if cplx else "NT"
        for ta in tr:
            for tb in tr:
                m, n, k = 13, 7, 37
                A, _ = mat(*op_shape(ta, m, k), cplx)
                B, _ = mat(*op_shape(tb, k, n), cplx)
                key = "%s%s%s" % ("z" if cplx else "d", ta, tb)
                out["dd_" + key] = oracle.gemm_dd(ta, tb, A, B)
                out["plain_" + key] = oracle.gemm_plain(ta, tb, A, B)
                out["emu_" + key] = oracle.emu_gemm(ta, tb, A, B, 5)
                out["emuk_" + key] = oracle.emu_gemm(ta, tb, A, B, 4, kc=8 if cplx else 5)
                out["grow_" + key] = oracle.emu_gemm(ta, tb, A, B, 3, s_to=6)
                out["bal_" + key] = oracle.emu_gemm(ta, tb, A, B, 6, balanced=True)
                out["sub_" + key] = oracle.emu_gemm(ta, tb, A, B, 7, rows=[0, 12, 5], cols=[6, 1])
                hi, lo = oracle.emu_gemm_x2(ta, tb, A, B, 9)
                out["x2hi_" + key], out["x2lo_" + key] = hi, lo
                if cplx:
                    out["3m_" + key] = oracle.emu_zgemm3(ta, tb, A, B, 6)
                    out["3mb_" + key] = oracle.emu_zgemm3(ta, tb, A, B, 5, balanced=True)
    # alpha / beta with a padded C
    A, _ = mat(9, 11)
    B, _ = mat(11, 6)
    C, _ = mat(9, 6)
    out["ab_d"] = oracle.emu_gemm("N", "N", A, B, 6, alpha=-1.5, beta=0.25, C=C)
    Az, _ = mat(9, 11, True)
    Bz, _ = mat(11, 6, True)
    Cz, _ = mat(9, 6, True)
    out["ab_z"] = oracle.emu_gemm("N", "N", Az, Bz, 6, alpha=0.5 - 2j, beta=1j, C=Cz)
    out["ab_z3"] = oracle.emu_zgemm3("N", "N", Az, Bz, 6, alpha=0.5 - 2j, beta=1j, C=Cz)
    out["dd_ab"] = oracle.gemm_dd("N", "N", Az, Bz, alpha=2.0, beta=-1.0, C=Cz)
    # views of padded buffers
    Ap, _ = mat(10, 17, ld=23)
    Bp, _ = mat(17, 5, ld=31)
    out["ld"] = oracle.emu_gemm("N", "N", Ap, Bp, 7)
    # split and diagonal sums, ragged sizes, both digit kinds
    for cplx in (False, True):
        X, _ = mat(19, 29, cplx)
        for bal in (False, True):
            E, dig = oracle.split("A", "N", X, 7, balanced=bal)
            out["splitE_%d%d" % (cplx, bal)], out["splitD_%d%d" % (cplx, bal)] = E, dig
        Ea, da = oracle.split("A", "N", X, 5)
        Eb, db = oracle.split("B", "T", X, 5)
        S = oracle.diag_sums(da, db, 5, kc=6 if cplx else 3)
        out["diag_%d" % cplx] = np.stack(S) if cplx else S
    # empty and degenerate shapes
    A0, _ = mat(4, 0)
    B0, _ = mat(0, 3)
    out["k0"] = oracle.emu_gemm("N", "N", A0, B0, 4)
    out["k0dd"] = oracle.gemm_dd("N", "N", A0, B0)
    out["m1"] = oracle.emu_gemm("N", "N", mat(1, 5)[0], mat(5, 1)[0], 3)
    # zero rows, Inf/NaN, subnormals
    A = mat(6, 8)[0].copy(order="F")
    A[2, :] = 0.0
    A[3, 1] = np.inf
    A[4, 5] = np.nan
    A[5, :] = np.ldexp(A[5, :], -1060)
    B = mat(8, 4)[0]
    out["special"] = oracle.emu_gemm("N", "N", A, B, 6)
    out["special_bal"] = oracle.emu_gemm("N", "N", A, B, 6, balanced=True)
    out["special_split"] = oracle.split("A", "N", A, 9)[1]
    return out
'''

CHILD = CASES_SRC + r'''
import sys
res = cases()
np.savez(sys.argv[1], **{k: np.asarray(v) for k, v in res.items()})
print("sanitized oracle: %d results" % len(res), flush=True)
'''


def test_oracle_under_asan_ubsan(tmp_path):
    san = obuild.build(sanitize=True)
    runtime = obuild.asan_runtime()
    if not os.path.isabs(runtime) or not os.path.exists(runtime):
        pytest.skip("gcc has no ASan runtime here")
    env = dict(os.environ)
    env["OZ_ORACLE_LIB"] = san
    # the ASan runtime goes first; anything already preloaded stays
    env["LD_PRELOAD"] = runtime + ((" " + env["LD_PRELOAD"]) if env.get("LD_PRELOAD") else "")
    env["ASAN_OPTIONS"] = "detect_leaks=0:verify_asan_link_order=0:abort_on_error=0:exitcode=77"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1:exitcode=78"
    env["OMP_NUM_THREADS"] = "4"
    env["PYTHONPATH"] = ROOT + os.pathsep + env.get("PYTHONPATH", "")
    script = tmp_path / "child.py"
    script.write_text(CHILD)
    out = tmp_path / "san.npz"
    p = subprocess.run([sys.executable, str(script), str(out)], env=env, capture_output=True, text=True,
                       timeout=600, cwd=str(tmp_path))
    report = p.stdout[-3000:] + p.stderr[-6000:]
    assert p.returncode == 0, report
    assert "AddressSanitizer" not in p.stderr and "runtime error" not in p.stderr, report
    # the same calls on the regular build give the same bits
    ns = {}
    exec(compile(CASES_SRC, "cases", "exec"), ns)
    want = ns["cases"]()
    got = np.load(out)
    assert sorted(got.files) == sorted(want)
    for key, val in want.items():
        g, w = np.ascontiguousarray(got[key]), np.ascontiguousarray(val)
        assert g.shape == w.shape and g.dtype == w.dtype, key
        assert np.array_equal(g.view(np.uint8), w.view(np.uint8)), key
