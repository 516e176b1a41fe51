"""Pins of the oracle's double-double product (emu_gemm_x2), none of which
reuses its double-double step:

* integer inputs with enough slices that no pair is dropped: hi + lo is the
  exact product (82-bit values), real and complex, for every trans;
* general wide-range doubles, several INT32 chunks: hi + lo is the exact
  rational sum of the oracle's own anti-diagonal sums times 2^(E+F-7d), and hi
  is that sum correctly rounded (float() of a Fraction);
* beyond FP64: the error against the exact product keeps falling past s = 8,
  where the FP64 result stops improving."""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle.exact import exact_gemm


def _ints(rng, shape, bits, cplx=False):
    x = rng.integers(-2 ** (bits - 1), 2 ** (bits - 1), size=shape).astype(float)
    if cplx:
        x = x + 1j * rng.integers(-2 ** (bits - 1), 2 ** (bits - 1), size=shape).astype(float)
    return np.asfortranarray(x)


def _stored(ta, shape):
    return shape if ta == "N" else shape[::-1]


@pytest.mark.parametrize("ta,tb", [("N", "N"), ("T", "N"), ("N", "T"), ("T", "T")])
def test_integer_products_are_exact_real(ta, tb):
    rng = np.random.default_rng(ord(ta) + 3 * ord(tb))
    m, n, k = 5, 4, 13
    A = _ints(rng, _stored(ta, (m, k)), 40)
    B = _ints(rng, (k, n) if tb == "N" else (n, k), 40)
    hi, lo = oracle.emu_gemm_x2(ta, tb, A, B, 12)
    re, _ = exact_gemm(ta, tb, A, B)
    for i in range(m):
        for j in range(n):
            assert Fraction(hi[i, j]) + Fraction(lo[i, j]) == re[i][j]
    assert np.abs(lo).max() > 0  # the products need more than 53 bits


@pytest.mark.parametrize("ta,tb", [("N", "N"), ("C", "N"), ("T", "C")])
def test_integer_products_are_exact_complex(ta, tb):
    rng = np.random.default_rng(ord(ta) * 5 + ord(tb))
    m, n, k = 4, 3, 9
    A = _ints(rng, _stored(ta, (m, k)), 35, True)
    B = _ints(rng, (k, n) if tb == "N" else (n, k), 35, True)
    hi, lo = oracle.emu_gemm_x2(ta, tb, A, B, 12)
    re, im = exact_gemm(ta, tb, A, B)
    for i in range(m):
        for j in range(n):
            assert Fraction(hi[i, j].real) + Fraction(lo[i, j].real) == re[i][j]
            assert Fraction(hi[i, j].imag) + Fraction(lo[i, j].imag) == im[i][j]


@pytest.mark.parametrize("s,kc", [(3, 64), (7, 128), (10, 64), (14, 192)])
def test_sum_of_the_diagonal_sums_exact_and_hi_rounded(s, kc):
    rng = np.random.default_rng(s)
    m, n, k = 6, 5, 300
    A = np.asfortranarray(rng.standard_normal((m, k)) * np.exp2(rng.integers(-30, 31, size=(m, k))))
    B = np.asfortranarray(rng.standard_normal((k, n)) * np.exp2(rng.integers(-30, 31, size=(k, n))))
    hi, lo = oracle.emu_gemm_x2("N", "N", A, B, s, kc=kc)
    EA, dA = oracle.split("A", "N", A, s)
    FB, dB = oracle.split("B", "N", B, s)
    S = np.asarray(oracle.diag_sums(dA, dB, s, kc=kc))  # [chunk, d - 2, row, col]
    for i in range(m):
        for j in range(n):
            ex = sum(Fraction(int(S[c, d - 2, i, j])) * Fraction(2) ** (int(EA[i]) + int(FB[j]) - 7 * d)
                     for c in range(S.shape[0]) for d in range(2, s + 2))
            assert Fraction(hi[i, j]) + Fraction(lo[i, j]) == ex
            assert hi[i, j] == float(ex)


def test_error_falls_past_fp64():
    rng = np.random.default_rng(11)
    m, n, k = 4, 4, 40
    A = np.asfortranarray(rng.standard_normal((m, k)))
    B = np.asfortranarray(rng.standard_normal((k, n)))
    re, _ = exact_gemm("N", "N", A, B)
    scale = float(np.abs(A).max() * np.abs(B).max())

    def err(s):
        hi, lo = oracle.emu_gemm_x2("N", "N", A, B, s)
        return max(abs(float(Fraction(hi[i, j]) + Fraction(lo[i, j]) - re[i][j])) for i in range(m)
                   for j in range(n)) / scale

    e = {s: err(s) for s in (8, 10, 12, 14, 16)}
    assert e[8] > 1e-17 and e[10] < 1e-18 and e[12] < 1e-22 and e[14] < 1e-26
    assert e[16] < 1e-29
    for s in (8, 10, 12, 14):
        assert e[s + 2] < e[s] * 2.0 ** -10
