"""Pins of the scale-weighted error metric, on the CPU.

The metric gates every accuracy claim: eps = ||W o (C - C*)||_F / ||W o C*||_F
with W_ij = 1 / (max_l |op(A)_il| * max_l |op(B)_lj|) (for complex data the
max runs over real and imaginary parts, the quantity the scale exponent is
taken from).  Three oracle functions implement it: ``oracle.weighted_error``
(every reported error), ``oracle.select.weights`` (the row and column maxima
of op(A), op(B)) and ``oracle.select.weighted_eps`` (the selector's labels).
Every expected value below is worked out by hand in the comments, so a
dropped weight, a swapped axis or an unweighted denominator fails here.
"""
import math

import numpy as np

import oracle
from oracle import select as osel


# Hand example, 2 x 3, distinct row and column maxima.
#   row maxima of op(A): a = (2, 4); column maxima of op(B): b = (1, 8, 1/2)
#   W = 1 / (a b^T) = [[1/2, 1/16, 1], [1/4, 1/32, 1/2]]
#   C* = [[2, 16, 1], [4, 32, 2]]   so   W o C* = all ones, ||.||_F = sqrt(6)
#   C - C* = [[0, 0, 0], [0, 0, 1]] so   W o (C - C*) has one entry 1/2
#   eps = (1/2) / sqrt(6)
ROWMAX = np.array([2.0, 4.0])
COLMAX = np.array([1.0, 8.0, 0.5])
CREF = np.array([[2.0, 16.0, 1.0], [4.0, 32.0, 2.0]])
CX = CREF + np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
WANT = 0.5 / math.sqrt(6.0)


def test_weighted_error_hand_value():
    assert math.isclose(oracle.weighted_error(CX, CREF, ROWMAX, COLMAX), WANT, rel_tol=1e-15)


def test_weighted_eps_hand_value():
    wa, wb = 1.0 / ROWMAX, 1.0 / COLMAX
    assert math.isclose(osel.weighted_eps(CX, CREF, wa, wb), WANT, rel_tol=1e-15)


def test_weighted_error_denominator_is_weighted():
    # unweighted denominator: ||C*||_F = sqrt(4 + 256 + 1 + 16 + 1024 + 4) = sqrt(1305)
    # would give (1/2) / sqrt(1305), 14.7x smaller than the weighted value
    got = oracle.weighted_error(CX, CREF, ROWMAX, COLMAX)
    assert not math.isclose(got, 0.5 / math.sqrt(1305.0), rel_tol=1e-3)
    # an unweighted numerator: 1 / sqrt(6) -- twice the weighted value
    assert not math.isclose(got, 1.0 / math.sqrt(6.0), rel_tol=1e-3)


def test_weighted_error_row_and_column_roles():
    # square 2 x 2 with row maxima (1, 4) and column maxima (2, 1/2):
    #   W = [[1/2, 2], [1/8, 1/2]]; the error sits at (0, 1) where W = 2,
    #   while its transpose position (1, 0) has W = 1/8.
    #   C* = [[2, 1/2], [8, 2]] -> W o C* = all ones, ||.|| = 2
    #   C - C* = [[0, 3], [0, 0]] -> W o dC = 6 at (0, 1) -> eps = 3
    #   with the roles swapped (W' = 1/(b a^T)): W' = [[1/2, 1/8], [2, 1/2]],
    #   W' o C* = [[1, 1/16], [16, 1]], W' o dC = 3/8: a very different value
    a, b = np.array([1.0, 4.0]), np.array([2.0, 0.5])
    Cref = np.array([[2.0, 0.5], [8.0, 2.0]])
    dC = np.array([[0.0, 3.0], [0.0, 0.0]])
    assert math.isclose(oracle.weighted_error(Cref + dC, Cref, a, b), 3.0, rel_tol=1e-15)
    assert math.isclose(osel.weighted_eps(Cref + dC, Cref, 1.0 / a, 1.0 / b), 3.0, rel_tol=1e-15)


def test_weighted_vs_plain_known_factor():
    # rows of C* differ by 100x; the weights equalise them.
    #   a = (1, 100), b = (1, 1): W = [[1, 1], [1/100, 1/100]], W o C* = all ones (norm 2)
    #   dC = delta at (0, 0): weighted eps = delta / 2
    #   plain Frobenius error = delta / sqrt(1 + 1 + 10^4 + 10^4) = delta / sqrt(20002)
    #   ratio weighted / plain = sqrt(20002) / 2
    delta = 2.0 ** -30  # 1 + delta is exact, so dC is exactly delta
    Cref = np.array([[1.0, 1.0], [100.0, 100.0]])
    dC = np.array([[delta, 0.0], [0.0, 0.0]])
    w = oracle.weighted_error(Cref + dC, Cref, np.array([1.0, 100.0]), np.array([1.0, 1.0]))
    plain = np.linalg.norm(dC) / np.linalg.norm(Cref)
    assert math.isclose(w, delta / 2.0, rel_tol=1e-12)
    assert math.isclose(w / plain, math.sqrt(20002.0) / 2.0, rel_tol=1e-12)
    # equal weights everywhere: weighted == plain
    w1 = oracle.weighted_error(Cref + dC, Cref, np.array([3.0, 3.0]), np.array([0.5, 0.5]))
    assert math.isclose(w1, plain, rel_tol=1e-12)


def test_weighted_error_complex_hand_value():
    # complex entries: |W o dC|^2 sums squared moduli.
    #   a = (1,), b = (2, 4): W = [[1/2, 1/4]]
    #   C* = [[2i, 4]] -> W o C* = [[i, 1]], norm sqrt(2)
    #   dC = [[3 + 4i, 0]] -> |W o dC| = 5/2 -> eps = (5/2) / sqrt(2)
    Cref = np.array([[2j, 4.0 + 0j]])
    dC = np.array([[3.0 + 4.0j, 0.0]])
    a, b = np.array([1.0]), np.array([2.0, 4.0])
    want = 2.5 / math.sqrt(2.0)
    assert math.isclose(oracle.weighted_error(Cref + dC, Cref, a, b), want, rel_tol=1e-15)
    assert math.isclose(osel.weighted_eps(Cref + dC, Cref, 1.0 / a, 1.0 / b), want, rel_tol=1e-15)


def test_weighted_error_zero_reference():
    # C* = 0: the unnormalised weighted norm is returned (no division by zero)
    got = oracle.weighted_error(np.array([[3.0, 4.0]]), np.zeros((1, 2)), np.array([1.0]), np.array([1.0, 1.0]))
    assert got == 5.0
    got2 = osel.weighted_eps(np.array([[3.0, 4.0]]), np.zeros((1, 2)), np.ones(1), np.ones(2))
    assert got2 == 5.0


def test_select_weights_rows_and_columns():
    # A (2 x 3): row maxima (4, 3), column maxima (1, 4, 3)
    A = np.array([[1.0, -4.0, 2.0], [0.5, 0.0, -3.0]], order="F")
    # B (3 x 2): column maxima (8, 1), row maxima (2, 0, 8)
    B = np.array([[2.0, -1.0], [0.0, 0.0], [8.0, 0.25]], order="F")
    wa, wb = osel.weights("N", "N", A, B)
    assert np.array_equal(wa, [1 / 4, 1 / 3]) and np.array_equal(wb, [1 / 8, 1.0])
    # transposed operands: rows of op(A) = columns of A, columns of op(B) = rows of B
    wa, wb = osel.weights("T", "T", A.T.copy(order="F"), B.T.copy(order="F"))
    assert np.array_equal(wa, [1 / 4, 1 / 3]) and np.array_equal(wb, [1 / 8, 1.0])
    wa, wb = osel.weights("T", "T", A, B)
    # op(A) = A^T (3 x 2): its rows are A's columns, maxima (1, 4, 3);
    # op(B) = B^T (2 x 3): its columns are B's rows, maxima (2, 0, 8) -> weight 0 for the zero row
    assert np.array_equal(wa, [1.0, 1 / 4, 1 / 3]) and np.array_equal(wb, [1 / 2, 0.0, 1 / 8])


def test_select_weights_complex_parts():
    # complex: the max runs over real and imaginary parts separately, not the modulus:
    # 3 + 4i contributes 4 (|z| would be 5)
    A = np.array([[3.0 + 4.0j, 1.0 - 2.0j]], order="F")
    B = np.array([[0.5 - 6.0j], [-7.0 + 1.0j]], order="F")
    wa, wb = osel.weights("N", "N", A, B)
    assert np.array_equal(wa, [1 / 4]) and np.array_equal(wb, [1 / 7])
    # conjugate transpose changes no magnitude
    wa2, wb2 = osel.weights("C", "C", A.conj().T.copy(order="F"), B.conj().T.copy(order="F"))
    assert np.array_equal(wa2, wa) and np.array_equal(wb2, wb)


def test_weights_feed_weighted_error_consistently():
    # the two implementations of the metric agree on random data with wide scalings
    rng = np.random.default_rng(5)
    A = rng.standard_normal((7, 9)) * 10.0 ** rng.integers(-6, 7, size=(7, 1))
    B = rng.standard_normal((9, 5)) * 10.0 ** rng.integers(-6, 7, size=(1, 5))
    C = A @ B
    Cx = C * (1 + 1e-10 * rng.standard_normal(C.shape))
    wa, wb = osel.weights("N", "N", A, B)
    e1 = osel.weighted_eps(Cx, C, wa, wb)
    e2 = oracle.weighted_error(Cx, C, np.abs(A).max(1), np.abs(B).max(0))
    assert math.isclose(e1, e2, rel_tol=1e-12)
