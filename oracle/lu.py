"""Oracle of the LU-based complex inversion with emulated trailing products.

TEST INFRASTRUCTURE ONLY (imported by tests and the benchmark's CPU leg).

The paper's application inverts complex matrices by LU (Sec. 3.2: the main
solver of the LSMS case is an LU-based matrix inverse, rich in ZGEMM), with
every ZGEMM emulated at the chosen split number.  This module is the plain
blocked algorithm, step by step, with every level-3 product done by the
oracle's emulated GEMM (``oracle.emu_gemm``) and all other arithmetic written
out on real and imaginary parts as separate FP64 operations (no fused
multiply-add):

getrf(A, nb, s)   right-looking LU with partial pivoting, panel by panel:
  * panel (nb columns): for each column j, the pivot is the first row of
    largest |re| + |im| at or below j; the rows j and pivot are swapped across
    the panel; the entries below the diagonal are multiplied by the pivot's
    reciprocal (pr - i pi) / (pr^2 + pi^2); the panel columns right of j get
    the rank-1 update a_rk - l_rj u_jk;
  * the panel's interchanges applied to the columns left and right of it, in
    order;
  * U12 <- L11^-1 A12 by forward substitution (unit lower, sums in index
    order);
  * A22 <- A22 - L21 U12 as an emulated product (alpha = -1, beta = 1).
getri(LU, piv, nb, s)   X = A^-1 by solving A X = I:
  * X <- P I (the interchanges in order);
  * forward, block row i: X_i <- X_i - L[i, :i] X[:i] (emulated), then
    X_i <- L_ii^-1 X_i;
  * backward, block row i from the last: X_i <- X_i - U[i, i+1:] X[i+1:]
    (emulated), then X_i <- U_ii^-1 X_i by back substitution: rows from the
    last, each row's sum taking the solved unknowns in the order they were
    solved (highest index first), then multiplied by the reciprocal of its
    diagonal entry.

A singular U (a zero pivot) is reported as info = j + 1 for the first such
column, as LAPACK does; the factorization then skips the scaling of that
column.  Pivot indices are 0-based global row numbers.
"""
import numpy as np

from . import emu_gemm


def _recip(pr, pi):
    d = pr * pr + pi * pi
    return pr / d, -pi / d


def _cmul(ar, ai, br, bi):
    return ar * br - ai * bi, ar * bi + ai * br


def _panel(Re, Im, j0, nb, piv, info):
    n = Re.shape[0]
    for c in range(nb):
        j = j0 + c
        mag = np.abs(Re[j:, j]) + np.abs(Im[j:, j])
        p = j + int(np.argmax(mag))
        piv[j] = p
        if p != j:
            for X in (Re, Im):
                tmp = X[j, j0:j0 + nb].copy()
                X[j, j0:j0 + nb] = X[p, j0:j0 + nb]
                X[p, j0:j0 + nb] = tmp
        pr, pi = Re[j, j], Im[j, j]
        if pr == 0.0 and pi == 0.0:
            if info[0] == 0:
                info[0] = j + 1
        else:
            rr, ri = _recip(pr, pi)
            lr, li = _cmul(Re[j + 1:, j], Im[j + 1:, j], rr, ri)
            Re[j + 1:, j], Im[j + 1:, j] = lr, li
        for k in range(j + 1, j0 + nb):
            ur, ui = Re[j, k], Im[j, k]
            tr, ti = _cmul(Re[j + 1:, j], Im[j + 1:, j], ur, ui)
            Re[j + 1:, k] = Re[j + 1:, k] - tr
            Im[j + 1:, k] = Im[j + 1:, k] - ti
    return n


def _swap_rows(Re, Im, rows, piv, cols):
    for j in rows:
        p = piv[j]
        if p != j:
            for X in (Re, Im):
                tmp = X[j, cols].copy()
                X[j, cols] = X[p, cols]
                X[p, cols] = tmp


def _trsm_lower_unit(Lr, Li, Br, Bi):
    """B <- L^-1 B, L unit lower (nb x nb); rows in order, sums in index order."""
    nb = Lr.shape[0]
    for i in range(nb):
        accr, acci = Br[i].copy(), Bi[i].copy()
        for k in range(i):
            tr, ti = _cmul(Lr[i, k], Li[i, k], Br[k], Bi[k])
            accr, acci = accr - tr, acci - ti
        Br[i], Bi[i] = accr, acci


def _trsm_upper(Ur, Ui, Br, Bi):
    """B <- U^-1 B, U upper (nb x nb); rows from the last, each sum over the
    solved unknowns in solve order (k = nb-1 down to i+1)."""
    nb = Ur.shape[0]
    for i in range(nb - 1, -1, -1):
        accr, acci = Br[i].copy(), Bi[i].copy()
        for k in range(nb - 1, i, -1):
            tr, ti = _cmul(Ur[i, k], Ui[i, k], Br[k], Bi[k])
            accr, acci = accr - tr, acci - ti
        rr, ri = _recip(Ur[i, i], Ui[i, i])
        Br[i], Bi[i] = _cmul(accr, acci, rr, ri)


def _emu_update(C, A, B, s, kc, balanced=False):
    """C <- C - A B as the emulated product (alpha = -1, beta = 1)."""
    return emu_gemm("N", "N", np.asfortranarray(A), np.asfortranarray(B), s, alpha=-1.0, beta=1.0,
                    C=np.asfortranarray(C), kc=kc, balanced=balanced)


def getrf(A, nb, s, kc=None, balanced=False):
    """LU with partial pivoting of the square complex A; returns (LU, piv, info).
    balanced: the emulated products take balanced digits."""
    A = np.asarray(A, dtype=np.complex128)
    n = A.shape[0]
    Re, Im = A.real.copy(), A.imag.copy()
    piv = np.arange(n)
    info = [0]
    for j0 in range(0, n, nb):
        b = min(nb, n - j0)
        _panel(Re, Im, j0, b, piv, info)
        rows = range(j0, j0 + b)
        if j0 > 0:
            _swap_rows(Re, Im, rows, piv, slice(0, j0))
        if j0 + b < n:
            _swap_rows(Re, Im, rows, piv, slice(j0 + b, n))
            sl, sr = slice(j0, j0 + b), slice(j0 + b, n)
            _trsm_lower_unit(Re[sl, sl], Im[sl, sl], Re[sl, sr], Im[sl, sr])
            below = slice(j0 + b, n)
            C = Re[below, sr] + 1j * Im[below, sr]
            L21 = Re[below, sl] + 1j * Im[below, sl]
            U12 = Re[sl, sr] + 1j * Im[sl, sr]
            C = _emu_update(C, L21, U12, s, kc, balanced)
            Re[below, sr], Im[below, sr] = C.real, C.imag
    return np.asfortranarray(Re + 1j * Im), piv, info[0]


def getri(LU, piv, nb, s, kc=None, balanced=False):
    """Inverse of the matrix whose factorization getrf returned."""
    LU = np.asarray(LU, dtype=np.complex128)
    n = LU.shape[0]
    Lr, Li = LU.real, LU.imag
    Xr = np.eye(n)
    Xi = np.zeros((n, n))
    _swap_rows(Xr, Xi, range(n), piv, slice(0, n))
    blocks = [(j0, min(nb, n - j0)) for j0 in range(0, n, nb)]
    for j0, b in blocks:  # forward: L Y = P I
        sl = slice(j0, j0 + b)
        if j0 > 0:
            C = Xr[sl] + 1j * Xi[sl]
            C = _emu_update(C, LU[sl, :j0], Xr[:j0] + 1j * Xi[:j0], s, kc, balanced)
            Xr[sl], Xi[sl] = C.real, C.imag
        _trsm_lower_unit(Lr[sl, sl], Li[sl, sl], Xr[sl], Xi[sl])
    for j0, b in reversed(blocks):  # backward: U X = Y
        sl = slice(j0, j0 + b)
        if j0 + b < n:
            C = Xr[sl] + 1j * Xi[sl]
            C = _emu_update(C, LU[sl, j0 + b:], Xr[j0 + b:] + 1j * Xi[j0 + b:], s, kc, balanced)
            Xr[sl], Xi[sl] = C.real, C.imag
        _trsm_upper(Lr[sl, sl], Li[sl, sl], Xr[sl], Xi[sl])
    return np.asfortranarray(Xr + 1j * Xi)
