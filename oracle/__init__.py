"""CPU oracle for the Ozaki-scheme INT8 emulation of DGEMM / ZGEMM.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg import this package; the product library never does, and the
oracle never imports the product.  It shares no code with the GPU path: the
arithmetic lives in ``oz_oracle.c`` (plain C, built by ``oracle/build.py``)
and ``exact.py`` (rational arithmetic); this module only marshals numpy arrays.

Functions (every array is a numpy array in column-major / Fortran order,
float64 or complex128; ``trans`` is 'N', 'T' or 'C'):

* ``gemm_plain``  O1: FP64 GEMM, plain dot products in index order.
* ``gemm_dd``     O2: double-double (Dot2) GEMM, rounded once; the accuracy
                  reference every error report uses.
* ``split``       the per-vector scale exponent and the s INT8 digits
                  (Sec. 2.2: matrices are split into low-precision slices).
* ``diag_sums``   the exact integer anti-diagonal sums S_{d,chunk}.
* ``emu_gemm``    the full emulated product: digits, pair products with
                  p + q <= s + 1, FP64 accumulation, alpha/beta.
* ``emu_zgemm3``  the complex product as three real emulated products (3M).
* ``emu_gemm_x2`` the emulated product with a double-double result.
* ``split(..., balanced=True)`` / ``emu_gemm(..., balanced=True)``: the
                  round-to-nearest (balanced) digits and their product.
* ``kchunk``      the INT32 chunk length (products per chunk).

Submodules ``select`` (features, error table and labels of the learned
slice-count selector) and ``mlp`` (the selector network: forward, pinball
loss, backward, Adam) are plain numpy; ``lu`` is the blocked LU factorisation
and inverse of a complex matrix with every level-3 update an ``emu_gemm``.

Parity of each function is pinned in tests/test_oracle_*.py; none is unpinned.
"""
import ctypes
import os

import numpy as np

from . import build as _build
from .exact import exact_gemm, exact_gemm_rounded  # noqa: F401

_lib = None

INT32_MAX = 2 ** 31 - 1
DIGIT_MAX = 127


def _load():
    global _lib
    if _lib is not None:
        return _lib
    path = os.environ.get("OZ_ORACLE_LIB")  # e.g. the sanitized build (oracle/build.py)
    if not path:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
    lib = ctypes.CDLL(path)
    I64, D, P, C = ctypes.c_int64, ctypes.c_double, ctypes.c_void_p, ctypes.c_char
    I32 = ctypes.c_int
    lib.oro_dgemm_plain.argtypes = [C, C, I64, I64, I64, D, P, I64, P, I64, D, P, I64]
    lib.oro_zgemm_plain.argtypes = [C, C, I64, I64, I64, P, P, I64, P, I64, P, P, I64]
    lib.oro_dgemm_dd.argtypes = [C, C, I64, I64, I64, D, P, I64, P, I64, D, P, I64, P, I64, P, I64, P, I64]
    lib.oro_zgemm_dd.argtypes = [C, C, I64, I64, I64, P, P, I64, P, I64, P, P, I64, P, I64, P, I64, P, I64]
    lib.oro_split.argtypes = [C, C, I32, I64, I64, P, I64, I32, P, P]
    lib.oro_split_bal.argtypes = [C, C, I32, I64, I64, P, I64, I32, P, P]
    lib.oro_emu_dgemm_bal.argtypes = [C, C, I64, I64, I64, D, P, I64, P, I64, D, P, I64, I32, I64,
                                      P, I64, P, I64, P, I64]
    lib.oro_emu_zgemm_bal.argtypes = [C, C, I64, I64, I64, P, P, I64, P, I64, P, P, I64, I32, I64,
                                      P, I64, P, I64, P, I64]
    lib.oro_diag_sums.argtypes = [I32, I32, I64, I64, P, I64, P, I64, P, I64, P, I64, P]
    lib.oro_emu_dgemm.argtypes = [C, C, I64, I64, I64, D, P, I64, P, I64, D, P, I64, I32, I32, I64,
                                  P, I64, P, I64, P, I64]
    lib.oro_emu_dgemm_x2.argtypes = [C, C, I64, I64, I64, P, I64, P, I64, I32, I64, P, I64, P, I64, P, P, I64]
    lib.oro_emu_zgemm_x2.argtypes = [C, C, I64, I64, I64, P, I64, P, I64, I32, I64, P, I64, P, I64, P, P, I64]
    lib.oro_emu_zgemm.argtypes = [C, C, I64, I64, I64, P, P, I64, P, I64, P, P, I64, I32, I32, I64,
                                  P, I64, P, I64, P, I64]
    lib.oro_num_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def num_threads():
    """OpenMP threads the oracle runs on."""
    return _load().oro_num_threads()


def _ptr(a):
    return None if a is None else a.ctypes.data


def _f(a, dtype):
    a = np.asarray(a, dtype=dtype)
    return np.asfortranarray(a)


def _dims(trans, X, side):
    """(rows, cols) of op(X): side 'A' gives (m, k), side 'B' gives (k, n)."""
    r, c = X.shape
    return (c, r) if trans.upper() in "TC" else (r, c)


def _sel(sel, n):
    if sel is None:
        return None, n
    s = np.ascontiguousarray(np.asarray(sel, dtype=np.int64))
    assert s.ndim == 1 and (s.size == 0 or (s.min() >= 0 and s.max() < n))
    return s, s.size


def _ld(X):
    return max(1, X.shape[0])


def kchunk(s, cplx=False, balanced=False):
    """INT32 chunk length in products per output entry.

    An anti-diagonal sum of one chunk holds at most s pair products per term
    (diagonal d = s + 1 has s pairs) and every pair product is at most 127^2 in
    magnitude (128^2 with balanced digits), so kc terms are safe while
    s * kc * 127^2 <= 2^31 - 1.  kc is rounded down to a multiple of 64; a
    complex entry consumes two products per value of l, so complex chunks cover
    kc / 2 values of l.
    """
    dmax = 128 if balanced else DIGIT_MAX
    kc = INT32_MAX // (s * dmax * dmax)
    kc -= kc % 64
    return int(kc)


def gemm_plain(transa, transb, A, B, alpha=1.0, beta=0.0, C=None):
    """O1: C = alpha*op(A)*op(B) + beta*C in plain FP64."""
    cplx = np.iscomplexobj(A) or np.iscomplexobj(B) or np.iscomplexobj(alpha) or np.iscomplexobj(beta)
    dt = np.complex128 if cplx else np.float64
    A, B = _f(A, dt), _f(B, dt)
    m, k = _dims(transa, A, "A")
    k2, n = _dims(transb, B, "B")
    assert k == k2
    Cout = np.zeros((m, n), dtype=dt, order="F") if C is None else _f(C, dt).copy(order="F")
    lib = _load()
    if cplx:
        al = np.array([complex(alpha).real, complex(alpha).imag])
        be = np.array([complex(beta).real, complex(beta).imag])
        lib.oro_zgemm_plain(transa.encode(), transb.encode(), m, n, k, _ptr(al), _ptr(A), _ld(A),
                            _ptr(B), _ld(B), _ptr(be), _ptr(Cout), max(1, m))
    else:
        lib.oro_dgemm_plain(transa.encode(), transb.encode(), m, n, k, float(alpha), _ptr(A), _ld(A),
                            _ptr(B), _ld(B), float(beta), _ptr(Cout), max(1, m))
    return Cout


def gemm_dd(transa, transb, A, B, alpha=1.0, beta=0.0, C=None, rows=None, cols=None):
    """O2: double-double GEMM on the selected rows x cols of C (all by default)."""
    cplx = np.iscomplexobj(A) or np.iscomplexobj(B) or np.iscomplexobj(alpha) or np.iscomplexobj(beta)
    dt = np.complex128 if cplx else np.float64
    A, B = _f(A, dt), _f(B, dt)
    m, k = _dims(transa, A, "A")
    k2, n = _dims(transb, B, "B")
    assert k == k2
    Cin = np.zeros((max(m, 1), max(n, 1)), dtype=dt, order="F") if C is None else _f(C, dt)
    rs, nr = _sel(rows, m)
    cs, nc = _sel(cols, n)
    out = np.zeros((nr, nc), dtype=dt, order="F")
    lib = _load()
    if cplx:
        al = np.array([complex(alpha).real, complex(alpha).imag])
        be = np.array([complex(beta).real, complex(beta).imag])
        lib.oro_zgemm_dd(transa.encode(), transb.encode(), m, n, k, _ptr(al), _ptr(A), _ld(A), _ptr(B),
                         _ld(B), _ptr(be), _ptr(Cin), _ld(Cin), _ptr(rs), nr, _ptr(cs), nc, _ptr(out),
                         max(1, nr))
    else:
        lib.oro_dgemm_dd(transa.encode(), transb.encode(), m, n, k, float(alpha), _ptr(A), _ld(A),
                         _ptr(B), _ld(B), float(beta), _ptr(Cin), _ld(Cin), _ptr(rs), nr, _ptr(cs), nc,
                         _ptr(out), max(1, nr))
    return out


def split(side, trans, X, s, balanced=False):
    """Scale exponents and digits of the vectors of one operand.

    side 'A': the vectors are the rows of op(X); side 'B': the columns of op(X).
    Returns (E, dig): E int32 [nv]; dig int8 [s, nv, k] for real data or
    [s, nv, k, 2] (real part, imaginary part) for complex data.  balanced:
    round-to-nearest digits (s <= 8), x = 2^(E'+1) sum_p d_p 2^(-8p) to half a
    unit of the last digit, with E' = E or E + 1 (the returned exponent; see
    oz_oracle.c); otherwise truncated base-128 digits, x = 2^E sum_p t_p 2^(-7p)
    up to the truncation residual.
    """
    assert not balanced or 1 <= s <= 8
    cplx = np.iscomplexobj(X)
    X = _f(X, np.complex128 if cplx else np.float64)
    if side == "A":
        nv, k = _dims(trans, X, "A")
    else:
        k, nv = _dims(trans, X, "B")
    E = np.zeros(nv, dtype=np.int32)
    shape = (s, nv, k, 2) if cplx else (s, nv, k)
    dig = np.zeros(shape, dtype=np.int8)
    fn = _load().oro_split_bal if balanced else _load().oro_split
    fn(side.encode(), trans.encode(), int(cplx), nv, k, _ptr(X), _ld(X), s, _ptr(E), _ptr(dig))
    return E, dig


def diag_sums(digA, digB, s, kc=None, rows=None, cols=None):
    """Exact anti-diagonal sums S[c, d-2, i, j] (d = 2..s+1) from split digits.

    digA, digB as returned by ``split``; complex digits give a pair (Sr, Si).
    kc is the chunk length in products (``kchunk`` by default).
    """
    cplx = digA.ndim == 4
    k = digA.shape[2]
    kc = kchunk(s, cplx) if kc is None else kc
    assert kc > 0 and (not cplx or kc % 2 == 0)
    nvA, nvB = digA.shape[1], digB.shape[1]
    lch = kc // 2 if cplx else kc
    nch = (k + lch - 1) // lch if k > 0 else 0
    rs, nr = _sel(rows, nvA)
    cs, nc = _sel(cols, nvB)
    planes = 2 if cplx else 1
    out = np.zeros(planes * nch * s * nc * nr, dtype=np.int64)
    dA = np.ascontiguousarray(digA)
    dB = np.ascontiguousarray(digB)
    _load().oro_diag_sums(int(cplx), s, k, kc, _ptr(dA), nvA, _ptr(dB), nvB, _ptr(rs), nr, _ptr(cs), nc,
                          _ptr(out))
    out = out.reshape(planes, nch, s, nc, nr).transpose(0, 1, 2, 4, 3)
    return (out[0], out[1]) if cplx else out[0]


def _op(trans, X):
    t = trans.upper()
    return X if t == "N" else (X.T if t == "T" else X.conj().T)


def emu_zgemm3(transa, transb, A, B, s, alpha=1.0, beta=0.0, C=None, kc=None, rows=None, cols=None,
               balanced=False, s_to=None):
    """O4, complex product in the 3-real-product form (3M).

    With op(A) = Ar + i Ai and op(B) = Br + i Bi, the pre-added operands
    As = Ar + Ai and Bs = Br + Bi are rounded once in FP64; the three real
    emulated products T1 = Ar Br, T2 = Ai Bi, T3 = As Bs (each with its own
    row / column scales, kc = ``kchunk(s)`` real terms) are combined as
    Cr = T1 - T2, Ci = (T3 - T1) - T2, and then alpha, beta are applied with
    the complex formula of the 4-product form (each product and sum rounded).
    balanced: the three real products take balanced digits (none of their
    operands is negated, so no digit of a negated value arises).
    s_to: each real product is formed at s and then grown to s_to by its
    top anti-diagonals (the incremental order of ``emu_gemm``); the three are
    combined once, at s_to."""
    A = _op(transa, _f(A, np.complex128))
    B = _op(transb, _f(B, np.complex128))
    Ar, Ai = np.asfortranarray(A.real), np.asfortranarray(A.imag)
    Br, Bi = np.asfortranarray(B.real), np.asfortranarray(B.imag)
    As = np.asfortranarray(Ar + Ai)
    Bs = np.asfortranarray(Br + Bi)
    kc = kchunk(s if s_to is None else s_to, balanced=balanced) if kc is None else kc
    T1 = emu_gemm("N", "N", Ar, Br, s, kc=kc, rows=rows, cols=cols, balanced=balanced, s_to=s_to)
    T2 = emu_gemm("N", "N", Ai, Bi, s, kc=kc, rows=rows, cols=cols, balanced=balanced, s_to=s_to)
    T3 = emu_gemm("N", "N", As, Bs, s, kc=kc, rows=rows, cols=cols, balanced=balanced, s_to=s_to)
    Cr = T1 - T2
    Ci = (T3 - T1) - T2
    xr, xi = complex(alpha).real, complex(alpha).imag
    yr, yi = complex(beta).real, complex(beta).imag
    outr = xr * Cr - xi * Ci
    outi = xr * Ci + xi * Cr
    if yr != 0.0 or yi != 0.0:
        m, n = A.shape[0], B.shape[1]
        C0 = _f(C, np.complex128) if C is not None else np.zeros((m, n), np.complex128, order="F")
        rs = np.arange(m) if rows is None else np.asarray(rows)
        cs = np.arange(n) if cols is None else np.asarray(cols)
        C0 = C0[np.ix_(rs, cs)]
        cr, ci = C0.real, C0.imag
        outr = outr + (yr * cr - yi * ci)
        outi = outi + (yr * ci + yi * cr)
    return np.asfortranarray(outr + 1j * outi)


def emu_gemm(transa, transb, A, B, s, alpha=1.0, beta=0.0, C=None, kc=None, rows=None, cols=None, s_to=None,
             balanced=False):
    """O4: the emulated GEMM on the selected rows x cols (all by default).

    s_to > s: start at s slices and grow one slice at a time to s_to, adding
    each new anti-diagonal last (the order of the incremental fallback); kc is
    then the chunk length of the s_to plan (``kchunk(s_to)`` by default).
    balanced: round-to-nearest digits and fold weights 2^(2-8d) (fixed s <= 8).
    """
    s1 = s if s_to is None else s_to
    assert s1 >= s
    assert not balanced or (s_to is None and 1 <= s <= 8)
    cplx = np.iscomplexobj(A) or np.iscomplexobj(B) or np.iscomplexobj(alpha) or np.iscomplexobj(beta)
    dt = np.complex128 if cplx else np.float64
    A, B = _f(A, dt), _f(B, dt)
    m, k = _dims(transa, A, "A")
    k2, n = _dims(transb, B, "B")
    assert k == k2
    kc = kchunk(s1, cplx, balanced) if kc is None else kc
    assert kc > 0 and (not cplx or kc % 2 == 0)
    Cin = np.zeros((max(m, 1), max(n, 1)), dtype=dt, order="F") if C is None else _f(C, dt)
    rs, nr = _sel(rows, m)
    cs, nc = _sel(cols, n)
    out = np.zeros((nr, nc), dtype=dt, order="F")
    lib = _load()
    if balanced and cplx:
        al = np.array([complex(alpha).real, complex(alpha).imag])
        be = np.array([complex(beta).real, complex(beta).imag])
        lib.oro_emu_zgemm_bal(transa.encode(), transb.encode(), m, n, k, _ptr(al), _ptr(A), _ld(A), _ptr(B),
                              _ld(B), _ptr(be), _ptr(Cin), _ld(Cin), s, kc, _ptr(rs), nr, _ptr(cs), nc,
                              _ptr(out), max(1, nr))
    elif balanced:
        lib.oro_emu_dgemm_bal(transa.encode(), transb.encode(), m, n, k, float(alpha), _ptr(A), _ld(A),
                              _ptr(B), _ld(B), float(beta), _ptr(Cin), _ld(Cin), s, kc, _ptr(rs), nr,
                              _ptr(cs), nc, _ptr(out), max(1, nr))
    elif cplx:
        al = np.array([complex(alpha).real, complex(alpha).imag])
        be = np.array([complex(beta).real, complex(beta).imag])
        lib.oro_emu_zgemm(transa.encode(), transb.encode(), m, n, k, _ptr(al), _ptr(A), _ld(A), _ptr(B),
                          _ld(B), _ptr(be), _ptr(Cin), _ld(Cin), s, s1, kc, _ptr(rs), nr, _ptr(cs), nc,
                          _ptr(out), max(1, nr))
    else:
        lib.oro_emu_dgemm(transa.encode(), transb.encode(), m, n, k, float(alpha), _ptr(A), _ld(A),
                          _ptr(B), _ld(B), float(beta), _ptr(Cin), _ld(Cin), s, s1, kc, _ptr(rs), nr,
                          _ptr(cs), nc, _ptr(out), max(1, nr))
    return out


def emu_gemm_x2(transa, transb, A, B, s, kc=None, rows=None, cols=None):
    """O4 beyond FP64: the product op(A) op(B) at s slices with its
    anti-diagonal sums folded into a double-double (d = s+1 down to 2, chunk
    by chunk; (hi, lo) + x by TwoSum, the error added to lo, then a fast
    TwoSum).  Returns (hi, lo), each scaled by 2^(E_i + F_j), on the selected
    rows x cols; hi + lo is the emulated sum while its terms span fewer than
    about 100 bits."""
    cplx = np.iscomplexobj(A) or np.iscomplexobj(B)
    dt = np.complex128 if cplx else np.float64
    A, B = _f(A, dt), _f(B, dt)
    m, k = _dims(transa, A, "A")
    k2, n = _dims(transb, B, "B")
    assert k == k2
    kc = kchunk(s, cplx) if kc is None else kc
    assert kc > 0 and (not cplx or kc % 2 == 0)
    rs, nr = _sel(rows, m)
    cs, nc = _sel(cols, n)
    hi = np.zeros((nr, nc), dtype=dt, order="F")
    lo = np.zeros((nr, nc), dtype=dt, order="F")
    lib = _load()
    fn = lib.oro_emu_zgemm_x2 if cplx else lib.oro_emu_dgemm_x2
    fn(transa.encode(), transb.encode(), m, n, k, _ptr(A), _ld(A), _ptr(B), _ld(B), s, kc, _ptr(rs), nr, _ptr(cs),
       nc, _ptr(hi), _ptr(lo), max(1, nr))
    return hi, lo


def weighted_error(Cx, Cref, A_rowmax, B_colmax):
    """Scale-weighted normwise relative error of Cx against Cref.

    Each entry is weighted by 1 / (max_l |op(A)_il| * max_l |op(B)_lj|), which
    removes wide row/column scalings; without them it is the plain
    Frobenius-norm relative error up to a few percent.
    """
    W = 1.0 / np.outer(A_rowmax, B_colmax)
    num = np.linalg.norm((W * (Cx - Cref)).ravel())
    den = np.linalg.norm((W * Cref).ravel())
    return float(num / den) if den > 0 else float(num)
