"""Pins of the LU-inversion oracle (oracle/lu.py) against what does not depend
on it: LAPACK's factorisation (same pivot rule), a textbook unblocked LU written
out here with exact rational arithmetic on tiny inputs, invariants of partial
pivoting, closed-form inverses (permutation, diagonal, identity), LAPACK's
singularity report, and the error of the inverse falling with the split number
(the trend of the paper's Table 1)."""
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg

from oracle import lu


def cmat(rng, n, m=None):
    m = n if m is None else m
    return np.asfortranarray(rng.standard_normal((n, m)) + 1j * rng.standard_normal((n, m)))


def perm_of(piv):
    """Row order P^T such that A[order] = L U (interchanges in order)."""
    order = np.arange(len(piv))
    for j, p in enumerate(piv):
        order[[j, p]] = order[[p, j]]
    return order


def split_lu(LU):
    L = np.tril(LU, -1) + np.eye(LU.shape[0])
    return L, np.triu(LU)


@pytest.mark.parametrize("n,nb", [(40, 8), (100, 32), (67, 16)])
def test_pivots_and_factors_match_lapack(n, nb):
    # LAPACK's zgetrf picks the first row of largest |re| + |im| too; at s = 14
    # the emulated updates are FP64-accurate, so pivots agree exactly and the
    # factors to rounding.
    rng = np.random.default_rng(100 + n)
    A = cmat(rng, n)
    LU, piv, info = lu.getrf(A, nb, 14)
    lu_ref, piv_ref = scipy.linalg.lu_factor(A)
    assert info == 0
    assert np.array_equal(piv, piv_ref)
    assert np.abs(LU - lu_ref).max() / np.abs(lu_ref).max() < 1e-13


@pytest.mark.parametrize("s", [3, 7, 14])
def test_reconstruction_and_pivot_bound(s):
    # P A = L U to the accuracy of the emulated updates; every multiplier
    # satisfies |l| <= sqrt(2) (|a| <= |re| + |im| <= |re p| + |im p| <= sqrt(2)|p|).
    rng = np.random.default_rng(7)
    n = 80
    A = cmat(rng, n)
    LU, piv, info = lu.getrf(A, 16, s)
    L, U = split_lu(LU)
    err = np.abs(A[perm_of(piv)] - L @ U).max() / np.abs(A).max()
    bound = {3: 1e-3, 7: 1e-10, 14: 1e-14}[s]
    assert err < bound
    assert np.abs(np.tril(LU, -1)).max() <= np.sqrt(2) * (1 + 1e-15)


def test_blocking_matches_textbook_lu_exactly_in_rationals():
    # Tiny integer matrix: the unblocked textbook LU with partial pivoting is
    # done here in exact complex rationals; the oracle's blocked LU (nb = 2,
    # ragged last panel) must give the same pivots and factors to rounding.
    rng = np.random.default_rng(3)
    n = 7
    A = np.asfortranarray(rng.integers(-9, 10, (n, n)) + 1j * rng.integers(-9, 10, (n, n)))
    M = [[(Fraction(int(A[i, j].real)), Fraction(int(A[i, j].imag))) for j in range(n)] for i in range(n)]
    piv = []
    for j in range(n):
        p = max(range(j, n), key=lambda r: (abs(M[r][j][0]) + abs(M[r][j][1]), -r))
        piv.append(p)
        M[j], M[p] = M[p], M[j]
        pr, pi = M[j][j]
        d = pr * pr + pi * pi
        for r in range(j + 1, n):
            ar, ai = M[r][j]
            lr, li = (ar * pr + ai * pi) / d, (ai * pr - ar * pi) / d
            M[r][j] = (lr, li)
            for c in range(j + 1, n):
                ur, ui = M[j][c]
                M[r][c] = (M[r][c][0] - (lr * ur - li * ui), M[r][c][1] - (lr * ui + li * ur))
    exact = np.array([[float(x[0]) + 1j * float(x[1]) for x in row] for row in M])
    LU, piv_o, info = lu.getrf(A, 2, 14)
    assert info == 0
    assert list(piv_o) == piv
    assert np.abs(LU - exact).max() < 1e-13 * np.abs(exact).max()


def test_closed_form_inverses():
    n = 9
    # identity: nothing to do, exact
    LU, piv, _ = lu.getrf(np.eye(n, dtype=complex), 4, 5)
    assert np.array_equal(lu.getri(LU, piv, 4, 5), np.eye(n))
    # permutation matrix: the pivots undo it; inverse is its transpose, exact
    rng = np.random.default_rng(11)
    P = np.eye(n, dtype=complex)[rng.permutation(n)]
    LU, piv, _ = lu.getrf(P, 4, 3)
    assert np.array_equal(lu.getri(LU, piv, 4, 3), P.T)
    # diagonal with power-of-two parts: every step is exact
    d = np.exp2(rng.integers(-20, 21, n)) * (1 + 1j * rng.integers(-1, 2, n))
    D = np.diag(d)
    LU, piv, _ = lu.getrf(D, 4, 2)
    assert np.array_equal(piv, np.arange(n))
    assert np.array_equal(lu.getri(LU, piv, 4, 2), np.diag(1 / d))


def test_singular_reports_first_zero_pivot():
    rng = np.random.default_rng(5)
    A = cmat(rng, 12)
    A[:, 5] = 0
    _, _, info = lu.getrf(A, 4, 7)
    _, info_ref = scipy.linalg.lapack.zgetrf(A)[1:]
    assert info == info_ref == 6


def test_inverse_residual_and_lapack_agreement():
    rng = np.random.default_rng(9)
    n = 96
    A = cmat(rng, n)
    LU, piv, _ = lu.getrf(A, 32, 14)
    X = lu.getri(LU, piv, 32, 14)
    assert np.abs(A @ X - np.eye(n)).max() < 1e-12
    Xr = np.linalg.inv(A)
    assert np.abs(X - Xr).max() / np.abs(Xr).max() < 1e-12


def test_inverse_error_falls_with_slices():
    # Each added slice carries 7 more bits of every operand, so the error of
    # the inverse drops by roughly 2^-7 per slice until FP64 rounding is reached.
    rng = np.random.default_rng(13)
    n = 64
    A = cmat(rng, n)
    Xr = np.linalg.inv(A)
    errs = []
    for s in (3, 4, 5, 6, 7):
        LU, piv, _ = lu.getrf(A, 16, s)
        X = lu.getri(LU, piv, 16, s)
        errs.append(np.abs(X - Xr).max() / np.abs(Xr).max())
    for a, b in zip(errs, errs[1:]):
        assert b < a / 20
    assert errs[-1] < 1e-10


def test_balanced_products_gain_about_one_bit_per_slice():
    # with balanced digits every one of the s slices carries one bit more, so
    # the inverse's error shrinks against truncated digits at the same s by a
    # factor near 2^(s-1), growing with s
    rng = np.random.default_rng(23)
    n = 64
    A = cmat(rng, n)
    Xr = np.linalg.inv(A)

    def err(s, bal):
        LU, piv, _ = lu.getrf(A, 16, s, balanced=bal)
        return np.abs(lu.getri(LU, piv, 16, s, balanced=bal) - Xr).max() / np.abs(Xr).max()

    gains = [err(s, False) / err(s, True) for s in (3, 4, 5, 6)]
    for s, g in zip((3, 4, 5, 6), gains):
        assert g >= 2 ** (s - 2), (s, g)
    assert gains == sorted(gains)

