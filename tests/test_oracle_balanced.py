"""Pins of the oracle's balanced (round-to-nearest) digits and their product
against what does not depend on it: exact rational arithmetic for the rounding
and the reconstruction, closed forms on small integers (where the first digit
is the integer itself and every other digit is zero), the s = 1 product written
out with plain rounding, the error decay per slice, the gain over truncated
digits at the same slice count, power-of-two equivariance and the INT32 chunk
bound with all-extreme digits."""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle.exact import exact_gemm_rounded


def rand_wide(rng, shape, span, cplx=False):
    x = rng.standard_normal(shape) * np.exp2(rng.integers(-span, span + 1, size=shape))
    if cplx:
        x = x + 1j * rng.standard_normal(shape) * np.exp2(rng.integers(-span, span + 1, size=shape))
    return np.asfortranarray(x)


def round_half_away(q):
    """Nearest integer to the Fraction q, ties away from zero."""
    a = abs(q)
    n = (a + Fraction(1, 2)).numerator // (a + Fraction(1, 2)).denominator
    return n if q >= 0 else -n


@pytest.mark.parametrize("s", [1, 2, 3, 5, 7, 8])
def test_digits_are_the_rounded_value_in_base_256(s):
    # x = 2^(E'+1) sum_p d_p 2^(-8p) must be the multiple of u = 2^(E'+1-8s)
    # nearest to x (ties away from zero), with d_2..d_s in [-128, 127] and
    # |d_1| <= 127; E' = E, or E + 1 when the row max M has M 2^(7-E) > 127
    rng = np.random.default_rng(s)
    X = rand_wide(rng, (6, 40), 30)
    X[0, :5] = [0.0, 2.0 ** -1070, -3 * 2.0 ** -1074, 1.5, -1.5]
    X[1, :4] = [1.0, -1.0, 2.0 ** -40, -(2.0 ** -40)]
    # exact ties: x / u = integer + 1/2
    X[2, 0] = 1.0
    # a row max with M 2^(7-E) > 127 (E' = E + 1) and one exactly at 127 (no bump)
    X[3:5, :] = np.ldexp(X[3:5, :], -40)
    X[3, 0] = 127.5 / 128
    X[4, 0] = -127.0 / 128
    E, dig = oracle.split("A", "N", X, s, balanced=True)
    for v in range(X.shape[0]):
        M = Fraction(float(np.max(np.abs(X[v]))))
        e = int(np.frexp(float(M))[1])
        assert int(E[v]) == (e + 1 if M * Fraction(2) ** (7 - e) > 127 else e)
        for l in range(X.shape[1]):
            x = Fraction(float(X[v, l]))
            d = [int(dig[p, v, l]) for p in range(s)]
            assert all(-128 <= t <= 127 for t in d[1:]) and abs(d[0]) <= 127
            N = sum(t * 256 ** (s - 1 - p) for p, t in enumerate(d))
            u = Fraction(2) ** (int(E[v]) + 1 - 8 * s)
            assert N == round_half_away(x / u), (v, l)
            assert abs(x - N * u) <= u / 2


def test_tie_rounds_away_from_zero():
    # row max 1.5 -> E = 1 (1.5 * 2^6 = 96 <= 127, no bump); s = 1:
    # N = round(|x| 2^6): 2^-7 gives 0.5 -> 1, -2^-7 gives -1, 3 * 2^-7 gives 1.5 -> 2
    X = np.array([[1.5, 2.0 ** -7, -(2.0 ** -7), 3 * 2.0 ** -7]])
    E, dig = oracle.split("A", "N", X, 1, balanced=True)
    assert E[0] == 1
    assert list(dig[0, 0]) == [96, 1, -1, 2]
    # row max 127.5 / 128 -> E = 0, 127.5 > 127: E' = 1 and N = round(|x| 2^6)
    E, dig = oracle.split("A", "N", np.array([[127.5 / 128, 1.0 / 256]]), 1, balanced=True)
    assert E[0] == 1
    assert list(dig[0, 0]) == [64, 0]


def test_small_integers_give_exact_products():
    # integer entries |x| <= 63 with every row / column max in [32, 64): E = 6
    # (M 2^(7-6) <= 126, no bump), N = 2x 256^(s-1), so d_1 = 2x and the rest
    # are zero -- the emulated product is the exact integer product at any s
    rng = np.random.default_rng(7)
    for s in (1, 3, 8):
        A = rng.integers(-63, 64, (20, 30)).astype(float)
        B = rng.integers(-63, 64, (30, 25)).astype(float)
        A[:, 0] = 40
        B[0, :] = -33
        E, dA = oracle.split("A", "N", A, s, balanced=True)
        assert np.all(E == 6) and np.array_equal(dA[0], 2 * A) and not dA[1:].any()
        assert np.array_equal(oracle.emu_gemm("N", "N", A, B, s, balanced=True), A @ B)
        Az = A + 1j * rng.integers(-63, 64, A.shape)
        Bz = B + 1j * rng.integers(-63, 64, B.shape)
        got = oracle.emu_gemm("N", "T", Az, np.asfortranarray(Bz.T), s, balanced=True)
        assert np.array_equal(got, Az @ Bz)


def test_one_slice_is_the_product_of_rounded_values():
    # s = 1: each entry becomes round(x 2^(7-E')) 2^(E'-7); the product is the
    # exact product of those values (small integers times powers of two)
    rng = np.random.default_rng(3)
    A = rand_wide(rng, (15, 20), 4)
    B = rand_wide(rng, (20, 12), 4)

    def rounded(X, axis):
        mx = np.max(np.abs(X), axis=axis, keepdims=True)
        E = np.frexp(mx)[1]
        E = E + (mx * np.exp2(7.0 - E) > 127)
        y = X * np.exp2(7.0 - E)
        return np.sign(y) * np.floor(np.abs(y) + 0.5) * np.exp2(E - 7.0)

    ref = rounded(A, 1) @ rounded(B, 0)
    assert np.array_equal(oracle.emu_gemm("N", "N", A, B, 1, balanced=True), ref)


def rel_err(C, R):
    return np.linalg.norm(C - R) / np.linalg.norm(R)


@pytest.mark.parametrize("cplx", [False, True])
def test_error_decay_and_gain_over_truncation(cplx):
    # each balanced slice carries 8 bits (truncated: 7): the error falls about
    # 2^8 per slice, and at the same s balanced digits beat truncated ones
    rng = np.random.default_rng(11)
    A = rand_wide(rng, (48, 64), 2, cplx)
    B = rand_wide(rng, (64, 40), 2, cplx)
    R = exact_gemm_rounded("N", "N", A, B)
    eb = [rel_err(oracle.emu_gemm("N", "N", A, B, s, balanced=True), R) for s in range(1, 7)]
    et = [rel_err(oracle.emu_gemm("N", "N", A, B, s), R) for s in range(1, 7)]
    for a, b in zip(eb[1:], eb[2:]):
        assert 2 ** 6.5 < a / b < 2 ** 9.5
    for s in range(2, 6):
        assert eb[s] < et[s] / 2


def test_power_of_two_equivariance():
    rng = np.random.default_rng(5)
    A = rand_wide(rng, (10, 16), 6)
    B = rand_wide(rng, (16, 9), 6)
    base = oracle.emu_gemm("N", "N", A, B, 6, balanced=True)
    r = np.exp2(rng.integers(-20, 21, 10))[:, None]
    c = np.exp2(rng.integers(-20, 21, 9))[None, :]
    got = oracle.emu_gemm("N", "N", A * r, B * c, 6, balanced=True)
    assert np.array_equal(got, base * r * c)
    # negation is not exact: the digits of -x are another base-256 form of -N
    # (d_2..d_s stay in [-128, 127]), so the dropped pairs p + q > s + 1 differ;
    # both results are within the error of the emulation
    neg = oracle.emu_gemm("N", "N", -A, B, 6, balanced=True)
    assert np.abs(neg + base).max() <= 1e-9 * np.abs(base).max()


@pytest.mark.parametrize("s", [1, 4, 8])
def test_chunk_bound_with_extreme_digits(s):
    kc = oracle.kchunk(s, balanced=True)
    assert kc % 64 == 0
    assert s * kc * 128 * 128 <= 2 ** 31 - 1 < s * (kc + 64) * 128 * 128
    # all digits -128 (x = -0.5 * 2^E * (1 + ...) pattern): one chunk of kc terms on
    # diagonal s + 1 reaches s * kc * 128^2 exactly in magnitude and stays in INT32
    d = np.full((s, 1, kc), -128, dtype=np.int8)
    S = oracle.diag_sums(d, d, s, kc=kc)
    assert S[0, s - 1, 0, 0] == s * kc * 128 * 128


@pytest.mark.parametrize("balanced", [False, True])
@pytest.mark.parametrize("ta", ["N", "C"])
def test_complex_is_the_real_product_over_two_k_terms(balanced, ta):
    # Re C is the real emulated product of the rows (ar, -ai) against (br, bi),
    # Im C that of (ar, ai) against (bi, br) (same shared scales; one INT32
    # chunk, so term order does not matter): the complex sums are pinned to the
    # real path, including the digits of the value -ai under balanced digits
    rng = np.random.default_rng(21)
    m, n, k = 24, 18, 40
    A = rand_wide(rng, (m, k), 3, True)
    B = rand_wide(rng, (k, n), 3, True)
    As = np.asfortranarray(A.conj().T) if ta == "C" else A
    for s in (2, 4, 7):
        got = oracle.emu_gemm(ta, "N", As, B, s, balanced=balanced)
        Ar, Ai, Br, Bi = A.real, A.imag, B.real, B.imag
        re = oracle.emu_gemm("N", "N", np.hstack([Ar, -Ai]), np.vstack([Br, Bi]), s, balanced=balanced)
        im = oracle.emu_gemm("N", "N", np.hstack([Ar, Ai]), np.vstack([Bi, Br]), s, balanced=balanced)
        assert np.array_equal(got.real, re) and np.array_equal(got.imag, im), s


def test_three_product_form_small_integers_exact():
    # 3M with balanced digits: parts |x| <= 63 (their sums <= 126, which need
    # no bump): every digit below the first is zero, so the complex product is
    # exact at any s
    rng = np.random.default_rng(17)
    A = rng.integers(-63, 64, (12, 20)) + 1j * rng.integers(-63, 64, (12, 20))
    B = rng.integers(-63, 64, (20, 9)) + 1j * rng.integers(-63, 64, (20, 9))
    for s in (1, 3, 8):
        got = oracle.emu_zgemm3("N", "N", np.asfortranarray(A), np.asfortranarray(B), s, balanced=True)
        assert np.array_equal(got, A @ B), s

