"""O3: exact rational GEMM with Python fractions (tiny inputs only).

Every finite double is a dyadic rational, so Fraction(x) is exact and the
product below is the exact value of alpha*op(A)*op(B) + beta*C.  float() of a
Fraction is correctly rounded (ties to even), so ``exact_gemm_rounded`` is the
correctly rounded FP64 result: the fixed point that O1 and O2 are checked
against.  Test infrastructure only.
"""
from fractions import Fraction

import numpy as np


def _op(X, trans):
    X = np.asarray(X)
    if trans.upper() == "N":
        return X
    if trans.upper() == "T":
        return X.T
    return X.conj().T


def _fr(z):
    """Exact (re, im) fractions of a real or complex scalar."""
    z = complex(z)
    return Fraction(z.real), Fraction(z.imag)


def exact_gemm(transa, transb, A, B, alpha=1.0, beta=0.0, C=None):
    """Exact result as two nested lists of Fractions (real part, imaginary part)."""
    oA, oB = _op(A, transa), _op(B, transb)
    m, k = oA.shape
    k2, n = oB.shape
    assert k == k2
    a = [[_fr(oA[i, l]) for l in range(k)] for i in range(m)]
    b = [[_fr(oB[l, j]) for j in range(n)] for l in range(k)]
    xr, xi = _fr(alpha)
    yr, yi = _fr(beta)
    re = [[Fraction(0)] * n for _ in range(m)]
    im = [[Fraction(0)] * n for _ in range(m)]
    for i in range(m):
        for j in range(n):
            sr, si = Fraction(0), Fraction(0)
            for l in range(k):
                ar, ai = a[i][l]
                br, bi = b[l][j]
                sr += ar * br - ai * bi
                si += ar * bi + ai * br
            rr, ri = xr * sr - xi * si, xr * si + xi * sr
            if C is not None and (yr != 0 or yi != 0):
                cr, ci = _fr(np.asarray(C)[i, j])
                rr += yr * cr - yi * ci
                ri += yr * ci + yi * cr
            re[i][j], im[i][j] = rr, ri
    return re, im


def exact_gemm_rounded(transa, transb, A, B, alpha=1.0, beta=0.0, C=None):
    """Correctly rounded FP64 (or complex128) value of the exact product."""
    re, im = exact_gemm(transa, transb, A, B, alpha, beta, C)
    cplx = np.iscomplexobj(A) or np.iscomplexobj(B) or np.iscomplexobj(alpha) or np.iscomplexobj(beta)
    m, n = len(re), (len(re[0]) if re else 0)
    if cplx:
        out = np.zeros((m, n), dtype=np.complex128)
        for i in range(m):
            for j in range(n):
                out[i, j] = complex(float(re[i][j]), float(im[i][j]))
    else:
        out = np.zeros((m, n), dtype=np.float64)
        for i in range(m):
            for j in range(n):
                out[i, j] = float(re[i][j])
    return out
