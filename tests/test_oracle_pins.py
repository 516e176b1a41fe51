"""Pins of the CPU oracle against facts fixed outside the oracle itself.

Each test checks the oracle against something it cannot agree with by
construction: exact rational arithmetic (every double is a dyadic rational),
closed forms, invariants of the splitting, special cases that reduce to a
textbook integer product, a-priori error bounds, and the per-slice error decay
printed in the paper's Table 1 (Sec. 4).
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import workloads
from oracle.exact import exact_gemm, exact_gemm_rounded

U = 2.0 ** -53
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rand_wide(rng, shape, span=60):
    return rng.standard_normal(shape) * np.exp2(rng.integers(-span, span + 1, size=shape))


def rand_cwide(rng, shape, span=60):
    return rand_wide(rng, shape, span) + 1j * rand_wide(rng, shape, span)


def frac_abs_sum(transa, transb, A, B):
    """sum_l |op(A)_il| |op(B)_lj| (real) or the complex analogue over the 2k real products."""
    def op(X, t):
        return X if t == "N" else (X.T if t == "T" else X.conj().T)
    a, b = op(np.asarray(A), transa), op(np.asarray(B), transb)
    if np.iscomplexobj(a) or np.iscomplexobj(b):
        a, b = a.astype(np.complex128), b.astype(np.complex128)
        return (np.abs(a.real) @ np.abs(b.real) + np.abs(a.imag) @ np.abs(b.imag),
                np.abs(a.real) @ np.abs(b.imag) + np.abs(a.imag) @ np.abs(b.real))
    return np.abs(a) @ np.abs(b)


# ---------------------------------------------------------------- O1 / O2 vs O3


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("ta,tb", [("N", "N"), ("T", "N"), ("N", "T"), ("T", "T")])
def test_dd_gemm_is_correctly_rounded_real(seed, ta, tb):
    rng = np.random.default_rng(seed)
    m, n, k = rng.integers(1, 7, size=3)
    A = rand_wide(rng, (m, k) if ta == "N" else (k, m))
    B = rand_wide(rng, (k, n) if tb == "N" else (n, k))
    C0 = rand_wide(rng, (m, n))
    alpha, beta = rand_wide(rng, (), 3), rand_wide(rng, (), 3)
    got = oracle.gemm_dd(ta, tb, A, B, alpha, beta, C0)
    want = exact_gemm_rounded(ta, tb, A, B, alpha, beta, C0)
    re, _ = exact_gemm(ta, tb, A, B, alpha, beta, C0)
    # Dot2 bound: |res - exact| <= u|exact| + gamma_{2k}^2 sum|terms| (terms incl. alpha, beta).
    absum = np.abs(alpha) * frac_abs_sum(ta, tb, A, B) + np.abs(beta) * np.abs(C0)
    g = 2 * (k + 2) * U
    for i in range(m):
        for j in range(n):
            err = abs(Fraction(float(got[i, j])) - re[i][j])
            assert err <= U * abs(re[i][j]) + Fraction(g * g * absum[i, j]) * 4
    # Without heavy cancellation the result is the correctly rounded value.
    assert np.array_equal(got, want) or np.max(np.abs(got - want) / np.abs(want)) <= 2 * U


def test_dd_gemm_cancellation_exact():
    # a.b = 1e-30 after cancelling terms of size 1: plain FP64 loses it all.
    A = np.array([[1.0, 1e-30, -1.0]])
    B = np.array([[1.0], [1.0], [1.0]])
    assert oracle.gemm_dd("N", "N", A, B)[0, 0] == 1e-30
    assert oracle.gemm_plain("N", "N", A, B)[0, 0] == 0.0


@pytest.mark.parametrize("seed", range(4))
def test_dd_gemm_complex_correctly_rounded(seed):
    rng = np.random.default_rng(100 + seed)
    m, n, k = rng.integers(1, 6, size=3)
    A = rand_cwide(rng, (k, m), 20)
    B = rand_cwide(rng, (k, n), 20)
    C0 = rand_cwide(rng, (m, n), 20)
    alpha, beta = complex(1.5, -0.25), complex(-0.5, 2.0)
    got = oracle.gemm_dd("C", "N", A, B, alpha, beta, C0)
    want = exact_gemm_rounded("C", "N", A, B, alpha, beta, C0)
    rel = np.maximum(np.abs(got.real - want.real) / np.abs(want.real),
                     np.abs(got.imag - want.imag) / np.abs(want.imag))
    assert np.max(rel) <= 2 * U


@pytest.mark.parametrize("seed", range(4))
def test_plain_gemm_within_textbook_bound(seed):
    rng = np.random.default_rng(200 + seed)
    m, n, k = 5, 4, 7
    A, B = rand_wide(rng, (m, k), 10), rand_wide(rng, (k, n), 10)
    got = oracle.gemm_plain("N", "N", A, B)
    re, _ = exact_gemm("N", "N", A, B)
    bound = (k * U / (1 - k * U)) * frac_abs_sum("N", "N", A, B)
    for i in range(m):
        for j in range(n):
            assert abs(Fraction(float(got[i, j])) - re[i][j]) <= Fraction(float(bound[i, j]))


# ---------------------------------------------------------------- splitting


def brute_exponent(vals):
    """Smallest E with max|x| < 2^E, searched over integers (0 for all zero)."""
    mx = max((abs(Fraction(float(v))) for v in vals), default=Fraction(0))
    if mx == 0:
        return 0
    E = -1100
    while not (mx < Fraction(2) ** E):
        E += 1
    return E


def brute_digit(x, E, p):
    """sign(x) * (floor(|x| 2^(7p - E)) mod 128), exact."""
    fx = Fraction(float(x))
    t = math.floor(abs(fx) * Fraction(2) ** (7 * int(p) - int(E))) % 128
    return -t if fx < 0 else t


def special_values():
    return np.array([0.0, -0.0, 1.0, -1.0, 0.5, 127.0 / 128, 2.0 ** -1074, -2.0 ** -1074, 2.0 ** -1022,
                     1.7976931348623157e308, 3.0 * 2.0 ** -1060, -1e-310, 1.0 - 2.0 ** -53,
                     2.0 ** 100, 1e-300])


@pytest.mark.parametrize("s", [1, 3, 7, 8, 12, 18])
def test_split_matches_exact_digits(s):
    rng = np.random.default_rng(s)
    rows = [rand_wide(rng, 9, 80), special_values(), rand_wide(rng, 9, 3) * 2.0 ** -1040,
            np.zeros(9), rand_wide(rng, 9, 2) * 2.0 ** 1000]
    for r in rows:
        X = np.asfortranarray(r.reshape(1, -1))
        E, dig = oracle.split("A", "N", X, s)
        assert E[0] == brute_exponent(r)
        for l, x in enumerate(r):
            for p in range(1, s + 1):
                assert dig[p - 1, 0, l] == brute_digit(x, E[0], p), (x, p)


@pytest.mark.parametrize("s", [1, 2, 5, 7, 8, 9, 13])
def test_reconstruction_invariant(s):
    rng = np.random.default_rng(7 + s)
    X = np.asfortranarray(rand_wide(rng, (6, 40), 12))
    E, dig = oracle.split("A", "N", X, s)
    for v in range(X.shape[0]):
        for l in range(X.shape[1]):
            x = Fraction(float(X[v, l]))
            rec = sum(Fraction(int(dig[p, v, l])) * Fraction(2) ** (int(E[v]) - 7 * (p + 1)) for p in range(s))
            res = x - rec
            # residual keeps the sign of x and is below one unit of the last digit
            assert res == 0 or (res > 0) == (x > 0)
            assert abs(res) < Fraction(2) ** (int(E[v]) - 7 * s)
            # exact once 7s >= 53 + gap, gap = E - frexp exponent of x
            if x != 0:
                gap = int(E[v]) - math.frexp(float(X[v, l]))[1]
                if 7 * s >= 53 + gap:
                    assert res == 0
            assert all(-127 <= int(dig[p, v, l]) <= 127 for p in range(s))


@pytest.mark.parametrize("trans", ["N", "T", "C"])
def test_split_vectors_follow_op(trans):
    rng = np.random.default_rng(3)
    X = np.asfortranarray(rand_cwide(rng, (5, 7), 8))
    opX = X if trans == "N" else (X.T if trans == "T" else X.conj().T)
    EA, dA = oracle.split("A", trans, X, 4)
    EB, dB = oracle.split("B", trans, X, 4)
    for v in range(opX.shape[0]):
        vals = np.concatenate([opX[v].real, opX[v].imag])
        assert EA[v] == brute_exponent(vals)
        for l in range(opX.shape[1]):
            assert dA[1, v, l, 0] == brute_digit(opX[v, l].real, EA[v], 2)
            assert dA[1, v, l, 1] == brute_digit(opX[v, l].imag, EA[v], 2)
    for v in range(opX.shape[1]):
        vals = np.concatenate([opX[:, v].real, opX[:, v].imag])
        assert EB[v] == brute_exponent(vals)
        for l in range(opX.shape[0]):
            assert dB[0, v, l, 1] == brute_digit(opX[l, v].imag, EB[v], 1)


# ---------------------------------------------------------------- INT32 bound


def test_int32_chunk_bound():
    # |digit| <= 127: one pair product is at most 16129; a k-term sum of one pair
    # stays in int32 iff k <= 133144 (16129 * 133144 = 2147479576 < 2^31).
    assert 16129 * 133144 <= 2 ** 31 - 1 < 16129 * 133145
    for s in range(1, 19):
        kc = oracle.kchunk(s)
        assert kc % 64 == 0 and kc > 0
        assert s * kc * 127 * 127 <= 2 ** 31 - 1
        assert s * (kc + 64) * 127 * 127 > 2 ** 31 - 1
    assert oracle.kchunk(1) == 133120 and oracle.kchunk(7) == 19008


def test_worst_case_digits_fit_int32():
    # every digit +127 on the largest diagonal at exactly kc terms: stays in int32
    s = 7
    kc = oracle.kchunk(s)
    k = kc
    dA = np.full((s, 1, k), 127, dtype=np.int8)
    dB = np.full((s, 1, k), 127, dtype=np.int8)
    S = oracle.diag_sums(dA, dB, s, kc=kc)
    assert S.shape == (1, s, 1, 1)
    assert S[0, s - 1, 0, 0] == s * k * 127 * 127 <= 2 ** 31 - 1
    assert S[0, 0, 0, 0] == k * 127 * 127  # d = 2: a single pair
    # one chunk more than that and the plan must split
    S2 = oracle.diag_sums(np.full((s, 1, k + 64), 127, np.int8), np.full((s, 1, k + 64), 127, np.int8), s, kc=kc)
    assert S2.shape[0] == 2 and S2[1, s - 1, 0, 0] == s * 64 * 127 * 127


# ---------------------------------------------------------------- closed forms


def test_integer_matrices_one_slice_is_integer_gemm():
    # |a| <= 127 with a row max in [64, 127] gives E = 7, so digit 1 is the entry
    # itself: s = 1 reproduces the textbook integer product exactly.
    rng = np.random.default_rng(11)
    m, n, k = 9, 8, 33
    A = rng.integers(-127, 128, size=(m, k)).astype(np.float64)
    B = rng.integers(-127, 128, size=(k, n)).astype(np.float64)
    A[:, 0] = 100.0
    B[0, :] = -77.0
    E, dA = oracle.split("A", "N", A, 1)
    F, dB = oracle.split("B", "N", B, 1)
    assert np.all(E == 7) and np.all(F == 7)
    S = oracle.diag_sums(dA, dB, 1)
    want = A.astype(np.int64) @ B.astype(np.int64)
    assert np.array_equal(S[0, 0], want)
    C = oracle.emu_gemm("N", "N", A, B, 1)
    assert np.array_equal(C, want.astype(np.float64))


@pytest.mark.parametrize("s", [2, 4, 7])
def test_identity_gives_truncated_operand(s):
    # A = I: row i of A has max 1, E = 1, digits (64, 0, ...) at column i only.
    # Then C = op(B) truncated to s digits under its column scales.
    rng = np.random.default_rng(s)
    n = 6
    B = np.asfortranarray(rand_wide(rng, (n, 5), 10))
    C = oracle.emu_gemm("N", "N", np.eye(n), B, s)
    for j in range(B.shape[1]):
        F = brute_exponent(B[:, j])
        for l in range(n):
            want = sum(Fraction(brute_digit(B[l, j], F, p)) * Fraction(2) ** (F - 7 * p) for p in range(1, s + 1))
            assert Fraction(float(C[l, j])) == want


def few_digit_matrix(rng, shape, ndig):
    """Entries with at most ndig nonzero base-128 digits under their vector scale
    (each vector holds an entry of magnitude in [64, 127] * 2^-7 so that E = 0)."""
    top = rng.integers(-127, 128, size=shape).astype(np.float64)
    val = np.ldexp(top, -7)
    for d in range(2, ndig + 1):
        val += np.ldexp(rng.integers(-127, 128, size=shape) * np.sign(top + (top == 0)), -7 * d)
    return val


@pytest.mark.parametrize("cplx", [False, True])
def test_exact_when_no_pair_is_dropped(cplx):
    # Digits p <= 2 only, s = 3: every nonzero pair has p + q <= 4 = s + 1, the
    # anti-diagonal sums are exact integers and acc needs < 53 bits, so the
    # emulation equals the exact product bit for bit.
    rng = np.random.default_rng(5)
    m, n, k = 7, 6, 9
    A = few_digit_matrix(rng, (m, k), 2)
    B = few_digit_matrix(rng, (k, n), 2)
    A[:, 0] = 100 / 128
    B[0, :] = 90 / 128
    if cplx:
        A = A + 1j * few_digit_matrix(rng, (m, k), 2)
        B = B + 1j * few_digit_matrix(rng, (k, n), 2)
    got = oracle.emu_gemm("N", "N", A, B, 3)
    want = exact_gemm_rounded("N", "N", A, B)
    assert np.array_equal(got, want)
    # one slice fewer drops nonzero pairs: not exact any more
    assert not np.array_equal(oracle.emu_gemm("N", "N", A, B, 2), want)
    # alpha and beta with few bits keep every product and sum exact as well
    C0 = few_digit_matrix(rng, (m, n), 2)
    if cplx:
        C0 = C0 + 1j * few_digit_matrix(rng, (m, n), 2)
        alpha, beta = complex(3, -2), complex(0.5, 1.5)
    else:
        alpha, beta = -3.0, 0.75
    got = oracle.emu_gemm("N", "N", A, B, 3, alpha=alpha, beta=beta, C=C0)
    assert np.array_equal(got, exact_gemm_rounded("N", "N", A, B, alpha, beta, C0))


# ---------------------------------------------------------------- a-priori bound


@pytest.mark.parametrize("s", [2, 3, 5, 7, 8])
@pytest.mark.parametrize("cplx", [False, True])
def test_a_priori_error_bound(s, cplx):
    # |C_emu - AB|_ij <= K 2^(E_i+F_j) ((s+2) 2^-7s + 1.01 s u) + u |AB|_ij with
    # K products per entry (k real, 2k complex): truncation leaves < 2^-7s per
    # scaled operand, dropped pairs add < 1.01 (s-1) 2^-7s, the s-term FP64 sum
    # adds < 1.01 s u times sum |a||b| 2^-(E+F) <= K.
    rng = np.random.default_rng(40 + s)
    m, n, k = 6, 5, 17
    A = rand_cwide(rng, (m, k), 15) if cplx else rand_wide(rng, (m, k), 15)
    B = rand_cwide(rng, (k, n), 15) if cplx else rand_wide(rng, (k, n), 15)
    E, _ = oracle.split("A", "N", A, 1)
    F, _ = oracle.split("B", "N", B, 1)
    got = oracle.emu_gemm("N", "N", A, B, s)
    re, im = exact_gemm("N", "N", A, B)
    K = 2 * k if cplx else k
    for i in range(m):
        for j in range(n):
            scale = Fraction(2) ** (int(E[i]) + int(F[j])) * K
            tol = scale * (Fraction(s + 2) * Fraction(2) ** (-7 * s) + Fraction(1.01) * s * Fraction(U))
            for part, ex in ((got[i, j].real, re[i][j]), (got[i, j].imag, im[i][j])):
                assert abs(Fraction(float(part)) - ex) <= tol + Fraction(U) * abs(ex)


# ---------------------------------------------------------------- equivariances


def test_power_of_two_scaling_equivariance():
    rng = np.random.default_rng(21)
    A, B = rand_wide(rng, (8, 12), 6), rand_wide(rng, (12, 7), 6)
    d1 = np.exp2(rng.integers(-9, 10, size=(8, 1)))
    d2 = np.exp2(rng.integers(-9, 10, size=(1, 7)))
    base = oracle.emu_gemm("N", "N", A, B, 5)
    scaled = oracle.emu_gemm("N", "N", d1 * A * 2.0 ** 3, 2.0 ** -5 * B * d2, 5)
    assert np.array_equal(scaled, d1 * base * d2 * 2.0 ** -2)


def test_sign_transpose_permutation():
    rng = np.random.default_rng(22)
    A, B = rand_wide(rng, (8, 12), 6), rand_wide(rng, (12, 7), 6)
    base = oracle.emu_gemm("N", "N", A, B, 6)
    assert np.array_equal(oracle.emu_gemm("N", "N", -A, B, 6), -base)
    assert np.array_equal(oracle.emu_gemm("N", "N", B.T.copy(), A.T.copy(), 6), base.T)
    assert np.array_equal(oracle.emu_gemm("T", "T", B, A, 6), base.T)
    perm = rng.permutation(8)
    assert np.array_equal(oracle.emu_gemm("N", "N", A[perm], B, 6), base[perm])
    kperm = rng.permutation(12)
    assert np.array_equal(oracle.emu_gemm("N", "N", A[:, kperm], B[kperm], 6), base)


def test_complex_with_zero_imaginary_equals_real():
    rng = np.random.default_rng(23)
    A, B = rand_wide(rng, (6, 9), 10), rand_wide(rng, (9, 5), 10)
    real = oracle.emu_gemm("N", "N", A, B, 5, alpha=1.25, beta=-0.5, C=np.ones((6, 5)))
    cpx = oracle.emu_gemm("N", "N", A.astype(complex), B.astype(complex), 5, alpha=1.25 + 0j,
                          beta=-0.5 + 0j, C=np.ones((6, 5), complex))
    assert np.array_equal(cpx.real, real) and np.all(cpx.imag == 0)


def test_conjugate_transpose_equals_explicit_copy():
    rng = np.random.default_rng(24)
    A, B = rand_cwide(rng, (9, 6), 10), rand_cwide(rng, (5, 9), 10)
    got = oracle.emu_gemm("C", "T", A, B, 6)
    want = oracle.emu_gemm("N", "N", A.conj().T.copy(), B.T.copy(), 6)
    assert np.array_equal(got, want)


def test_alpha_beta_semantics():
    rng = np.random.default_rng(25)
    A, B = rand_wide(rng, (6, 9), 10), rand_wide(rng, (9, 5), 10)
    v = oracle.emu_gemm("N", "N", A, B, 6)
    # alpha = 1, beta = 1, C = -v cancels exactly
    assert np.all(oracle.emu_gemm("N", "N", A, B, 6, alpha=1.0, beta=1.0, C=-v) == 0)
    # beta = 0 never reads C
    assert np.array_equal(oracle.emu_gemm("N", "N", A, B, 6, beta=0.0, C=np.full((6, 5), np.nan)), v)
    # power-of-two alpha is exact
    assert np.array_equal(oracle.emu_gemm("N", "N", A, B, 6, alpha=0.25), v * 0.25)
    # general alpha, beta: two rounded products and one rounded add
    C0 = rand_wide(rng, (6, 5), 4)
    got = oracle.emu_gemm("N", "N", A, B, 6, alpha=1.1, beta=-0.3, C=C0)
    assert np.array_equal(got, (1.1 * v) + (-0.3 * C0))


def test_chunking_only_changes_rounding():
    # integer data: every partial sum is exact, so any chunk length gives the same C
    rng = np.random.default_rng(26)
    A = rng.integers(-127, 128, size=(5, 300)).astype(np.float64)
    B = rng.integers(-127, 128, size=(300, 4)).astype(np.float64)
    full = oracle.emu_gemm("N", "N", A, B, 3)
    assert np.array_equal(full, oracle.emu_gemm("N", "N", A, B, 3, kc=64))
    assert np.array_equal(full, A @ B)
    # general data: chunked and unchunked differ by rounding only
    A, B = rand_wide(rng, (5, 300), 4), rand_wide(rng, (300, 4), 4)
    c1 = oracle.emu_gemm("N", "N", A, B, 7)
    c2 = oracle.emu_gemm("N", "N", A, B, 7, kc=64)
    assert np.max(np.abs(c1 - c2) / np.abs(oracle.gemm_dd("N", "N", A, B))) < 1e-12
    S = oracle.diag_sums(*[oracle.split(sd, "N", X, 7)[1] for sd, X in (("A", A), ("B", B))], 7, kc=64)
    assert S.shape[0] == 5  # ceil(300 / 64) chunks


# ---------------------------------------------------------------- error decay (Table 1)


def load_table1():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "table1_iter1_max_real.txt")) if not l.startswith("#")]
    return {int(s): float(v) for s, v in rows}


def test_error_decay_per_slice_matches_table1():
    # Table 1 (Sec. 4): each extra split cuts the error by about 2^6.6 until the
    # FP64 floor; s = 3, 4 are FP32-like, s = 7, 8 are at FP64 level.
    t1 = load_table1()
    paper_rate = (math.log2(t1[3]) - math.log2(t1[9])) / 6
    assert 6.0 < paper_rate < 7.2
    import workloads
    A, B = workloads.dgemm_uniform(128, 128, 128, seed=0)
    ref = oracle.gemm_dd("N", "N", A, B)
    amax = np.max(np.abs(A), axis=1)
    bmax = np.max(np.abs(B), axis=0)
    eps = {s: oracle.weighted_error(oracle.emu_gemm("N", "N", A, B, s), ref, amax, bmax) for s in range(3, 9)}
    for s in range(3, 7):
        rate = math.log2(eps[s] / eps[s + 1])
        assert abs(rate - paper_rate) < 1.0, (s, rate, paper_rate)
    assert 1e-8 < eps[3] < 1e-4          # FP32-like
    assert eps[7] <= 1e-12               # the FP64-equivalent target
    native = oracle.weighted_error(oracle.gemm_plain("N", "N", A, B), ref, amax, bmax)
    assert eps[8] < 10 * native          # s = 8 at the FP64 floor


# ---------------------------------------------------------------- incremental growth


@pytest.mark.parametrize("cplx", [False, True])
def test_incremental_growth_reduces_and_is_exact(cplx):
    rng = np.random.default_rng(31)
    A = rand_cwide(rng, (7, 20), 10) if cplx else rand_wide(rng, (7, 20), 10)
    B = rand_cwide(rng, (20, 6), 10) if cplx else rand_wide(rng, (20, 6), 10)
    # no growth: the plain emulation
    assert np.array_equal(oracle.emu_gemm("N", "N", A, B, 5, s_to=5), oracle.emu_gemm("N", "N", A, B, 5))
    # digits p <= 2 only: growing 2 -> 3 adds exactly the missing pairs (2,2),(1,3),(3,1)
    # (the latter two are zero), so the grown result is the exact product
    A2 = few_digit_matrix(rng, (7, 9), 2)
    B2 = few_digit_matrix(rng, (9, 6), 2)
    A2[:, 0], B2[0, :] = 100 / 128, 90 / 128
    if cplx:
        A2 = A2 + 1j * few_digit_matrix(rng, (7, 9), 2)
        B2 = B2 + 1j * few_digit_matrix(rng, (9, 6), 2)
    assert np.array_equal(oracle.emu_gemm("N", "N", A2, B2, 2, s_to=3), exact_gemm_rounded("N", "N", A2, B2))


@pytest.mark.parametrize("s0,s1", [(3, 4), (4, 7), (5, 9)])
def test_incremental_growth_equals_fresh_run_up_to_rounding(s0, s1):
    # the grown and the fresh s1 results add the same exact terms in different
    # orders: they differ by at most ~ (s1 + 1) u sum|terms| <= (s1 + 1) u K 2^(E+F)
    rng = np.random.default_rng(s0 * 10 + s1)
    A, B = rand_wide(rng, (9, 40), 8), rand_wide(rng, (40, 8), 8)
    E, _ = oracle.split("A", "N", A, 1)
    F, _ = oracle.split("B", "N", B, 1)
    grown = oracle.emu_gemm("N", "N", A, B, s0, s_to=s1)
    fresh = oracle.emu_gemm("N", "N", A, B, s1)
    bound = (s1 + 1) * U * 40 * np.exp2(E[:, None] + F[None, :].astype(float))
    assert np.all(np.abs(grown - fresh) <= bound)
    # and each growth step brings the error down like a fresh run would
    ref = oracle.gemm_dd("N", "N", A, B)
    amax, bmax = np.abs(A).max(1), np.abs(B).max(0)
    e0 = oracle.weighted_error(oracle.emu_gemm("N", "N", A, B, s0), ref, amax, bmax)
    e1 = oracle.weighted_error(grown, ref, amax, bmax)
    assert e1 < e0 * 2.0 ** (-5 * (s1 - s0)) or e1 < 1e-15


# ---------------------------------------------------------------- 3M complex form

def _int_complex(rng, shape, lim):
    return (rng.integers(-lim, lim + 1, shape) + 1j * rng.integers(-lim, lim + 1, shape)).astype(np.complex128)


def test_3m_exact_on_small_integers():
    """Parts in [-63, 63]: Ar, Ai, Ar + Ai, Br, Bi, Br + Bi are integers of at
    most 7 bits, so one slice represents each exactly and the three real
    products, their combination and the result are exact (k 127^2 << 2^53)."""
    rng = np.random.default_rng(31)
    A = _int_complex(rng, (23, 40), 63)
    B = _int_complex(rng, (40, 17), 63)
    want = (A.astype(np.complex128) @ B.astype(np.complex128))  # exact: integer sums below 2^53
    Ai = A.real.astype(np.int64), A.imag.astype(np.int64)
    Bi = B.real.astype(np.int64), B.imag.astype(np.int64)
    exact_r = Ai[0] @ Bi[0] - Ai[1] @ Bi[1]
    exact_i = Ai[0] @ Bi[1] + Ai[1] @ Bi[0]
    assert np.array_equal(want.real, exact_r) and np.array_equal(want.imag, exact_i)
    for s in (1, 3):
        got = oracle.emu_zgemm3("N", "N", np.asfortranarray(A), np.asfortranarray(B), s)
        assert np.array_equal(got.real, exact_r.astype(float)) and np.array_equal(got.imag, exact_i.astype(float))
    # complex alpha / beta on exact data: the epilogue formula, exact here
    C0 = _int_complex(rng, (23, 17), 9)
    got = oracle.emu_zgemm3("N", "N", np.asfortranarray(A), np.asfortranarray(B), 2, alpha=2 - 1j, beta=0.5 + 0.25j,
                            C=np.asfortranarray(C0))
    want = (2 - 1j) * (exact_r + 1j * exact_i) + (0.5 + 0.25j) * C0
    assert np.array_equal(got, want)


def test_3m_trans_conj_and_rows():
    rng = np.random.default_rng(32)
    A = np.asfortranarray(rng.standard_normal((30, 44)) + 1j * rng.standard_normal((30, 44)))
    B = np.asfortranarray(rng.standard_normal((44, 21)) + 1j * rng.standard_normal((44, 21)))
    ref = oracle.emu_zgemm3("N", "N", A, B, 5)
    # op() given by trans / conj-trans storage yields the same operands bit for bit
    assert np.array_equal(oracle.emu_zgemm3("C", "T", np.asfortranarray(A.conj().T), np.asfortranarray(B.T), 5), ref)
    # row / column subsets select entries
    rows, cols = [3, 0, 29], [20, 1]
    assert np.array_equal(oracle.emu_zgemm3("N", "N", A, B, 5, rows=rows, cols=cols), ref[np.ix_(rows, cols)])


def test_3m_error_decays_and_stays_near_4m():
    A, B = workloads.zgemm_rowexp(n=96, seed=5, m=80, k=120)
    dd = oracle.gemm_dd("N", "N", A, B)
    wa = np.maximum(np.abs(A.real), np.abs(A.imag)).max(1)
    wb = np.maximum(np.abs(B.real), np.abs(B.imag)).max(0)
    prev = None
    for s in (3, 4, 5, 6, 7):
        e3 = oracle.weighted_error(oracle.emu_zgemm3("N", "N", A, B, s), dd, wa, wb)
        e4 = oracle.weighted_error(oracle.emu_gemm("N", "N", A, B, s), dd, wa, wb)
        assert e4 / 2 <= e3 <= 4 * e4, (s, e3, e4)     # same order as the 4-product form
        if prev is not None:
            assert 2 ** 5 < prev / e3 < 2 ** 8.5, s        # about 2^6.6 per slice (Table 1)
        prev = e3
    assert prev < 1e-12


@pytest.mark.parametrize("s0,s1", [(2, 5), (4, 7)])
def test_3m_growth_matches_fresh_run_up_to_rounding(s0, s1):
    """The 3-product form grown from s0 to s1 (each real product by its top
    anti-diagonals, combined once): no growth is the plain form; each real
    product differs from a fresh s1 run only by the order of the same exact
    terms, (s1 + 1) u K 2^(E+F) at most, and the combine's two differences
    add those bounds plus their own roundings; the error falls with s."""
    rng = np.random.default_rng(70 + s0)
    A = rand_cwide(rng, (9, 40), 8)
    B = rand_cwide(rng, (40, 8), 8)
    assert np.array_equal(oracle.emu_zgemm3("N", "N", A, B, s0, s_to=s0), oracle.emu_zgemm3("N", "N", A, B, s0))
    grown = oracle.emu_zgemm3("N", "N", A, B, s0, s_to=s1)
    fresh = oracle.emu_zgemm3("N", "N", A, B, s1)
    parts_a = [A.real, A.imag, A.real + A.imag]
    parts_b = [B.real, B.imag, B.real + B.imag]
    bnd = []
    for pa, pb in zip(parts_a, parts_b):
        E, _ = oracle.split("A", "N", np.asfortranarray(pa), 1)
        F, _ = oracle.split("B", "N", np.asfortranarray(pb), 1)
        bnd.append((s1 + 1) * U * 40 * np.exp2(E[:, None] + F[None, :].astype(float)))
    mag = np.abs(fresh.real) + np.abs(fresh.imag)
    assert np.all(np.abs(grown.real - fresh.real) <= bnd[0] + bnd[1] + 4 * U * mag + 1e-300)
    assert np.all(np.abs(grown.imag - fresh.imag) <= bnd[0] + bnd[1] + bnd[2] + 8 * U * mag + 1e-300)
    ref = oracle.gemm_dd("N", "N", A, B)
    wa = np.maximum(np.abs(A.real), np.abs(A.imag)).max(1)
    wb = np.maximum(np.abs(B.real), np.abs(B.imag)).max(0)
    e0 = oracle.weighted_error(oracle.emu_zgemm3("N", "N", A, B, s0), ref, wa, wb)
    e1 = oracle.weighted_error(grown, ref, wa, wb)
    assert e1 < e0 * 2.0 ** (-5 * (s1 - s0)) or e1 < 1e-15
