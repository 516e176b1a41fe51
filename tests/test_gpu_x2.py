"""Products with a double-double result (oz_dgemm_x2 / oz_zgemm_x2) against
the oracle's emu_gemm_x2: high and low parts bit-exact, over trans cases,
padded leading dimensions, slice counts 2..18, forced INT32 chunks and
non-finite rows; at full size, sampled entries bit-exact and the error against
the exact product falling past FP64."""
from fractions import Fraction

import numpy as np
import pytest
import torch

import oracle
from gpu_util import from_dev, to_dev
from oracle.exact import exact_gemm

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def oz():
    import paper_2503_22875_amd as mod
    return mod


@pytest.fixture(scope="module")
def handle(oz):
    torch.cuda.set_device(0)
    h = oz.oz_create(0)
    oz.oz_set_stream(h, torch.cuda.current_stream().cuda_stream)
    yield h
    oz.oz_destroy(h)


def wide(rng, shape, span, cplx=False):
    x = rng.standard_normal(shape)
    if cplx:
        x = x + 1j * rng.standard_normal(shape)
    return np.asfortranarray(x * np.exp2(rng.integers(-span, span + 1, size=shape)))


def run_x2(oz, handle, ta, tb, A, B, s, kchunk=0, check=True):
    cplx = np.iscomplexobj(A)
    m = A.shape[0] if ta == "N" else A.shape[1]
    k = A.shape[1] if ta == "N" else A.shape[0]
    n = B.shape[1] if tb == "N" else B.shape[0]
    dA, lda = to_dev(A, A.shape[0] + 1)
    dB, ldb = to_dev(B, B.shape[0] + 2)
    zero = np.zeros((m, n), A.dtype, order="F")
    dH, ldc = to_dev(zero, m + 3)
    dL, _ = to_dev(zero, m + 3)
    fn = oz.oz_zgemm_x2 if cplx else oz.oz_dgemm_x2
    st, rep = fn(handle, ta, tb, m, n, k, dA, lda, dB, ldb, dH, dL, ldc, oz.prec(s, kchunk=kchunk), report=True,
                 check=check)
    torch.cuda.synchronize()
    return st, rep, from_dev(dH, m, n, ldc), from_dev(dL, m, n, ldc)


@pytest.mark.parametrize("s", [2, 7, 9, 12, 14, 18])
@pytest.mark.parametrize("ta,tb", [("N", "N"), ("T", "N"), ("N", "T"), ("T", "T")])
def test_dgemm_x2_bit_exact(oz, handle, s, ta, tb):
    rng = np.random.default_rng(100 * s + ord(ta) + 3 * ord(tb))
    m, n, k = 70, 65, 300
    A = wide(rng, (m, k) if ta == "N" else (k, m), 30)
    B = wide(rng, (k, n) if tb == "N" else (n, k), 30)
    print("x2 real", s, ta, tb, flush=True)
    st, rep, hi, lo = run_x2(oz, handle, ta, tb, A, B, s)
    whi, wlo = oracle.emu_gemm_x2(ta, tb, A, B, s)
    assert st == 0 and rep.status == 0
    assert np.array_equal(hi, whi) and np.array_equal(lo, wlo)


@pytest.mark.parametrize("s", [6, 11])
@pytest.mark.parametrize("ta,tb", [("N", "N"), ("C", "N"), ("T", "C"), ("C", "T")])
def test_zgemm_x2_bit_exact(oz, handle, s, ta, tb):
    rng = np.random.default_rng(7 * s + ord(ta) + 5 * ord(tb))
    m, n, k = 50, 40, 120
    A = wide(rng, (m, k) if ta == "N" else (k, m), 20, True)
    B = wide(rng, (k, n) if tb == "N" else (n, k), 20, True)
    print("x2 complex", s, ta, tb, flush=True)
    st, rep, hi, lo = run_x2(oz, handle, ta, tb, A, B, s)
    whi, wlo = oracle.emu_gemm_x2(ta, tb, A, B, s)
    assert np.array_equal(hi, whi) and np.array_equal(lo, wlo)


@pytest.mark.parametrize("cplx", [0, 1])
def test_x2_forced_chunks_and_exact_integers(oz, handle, cplx):
    rng = np.random.default_rng(3 + cplx)
    m, n, k = 33, 47, 700
    A = wide(rng, (m, k), 25, bool(cplx))
    B = wide(rng, (k, n), 25, bool(cplx))
    print("x2 chunks", cplx, flush=True)
    st, rep, hi, lo = run_x2(oz, handle, "N", "N", A, B, 10, kchunk=128)
    whi, wlo = oracle.emu_gemm_x2("N", "N", A, B, 10, kc=128)
    assert rep.kchunks > 1
    assert np.array_equal(hi, whi) and np.array_equal(lo, wlo)
    st, rep, hi, lo = run_x2(oz, handle, "N", "N", A, B, 12, kchunk=128)  # chunked at s = 12: streaming kernel
    whi, wlo = oracle.emu_gemm_x2("N", "N", A, B, 12, kc=128)
    assert rep.kchunks > 1
    assert np.array_equal(hi, whi) and np.array_equal(lo, wlo)
    # integer inputs at s = 12: hi + lo is the exact product (about 80 bits)
    Ai = np.asfortranarray(rng.integers(-2 ** 39, 2 ** 39, size=(9, 20)).astype(float))
    Bi = np.asfortranarray(rng.integers(-2 ** 39, 2 ** 39, size=(20, 7)).astype(float))
    st, rep, hi, lo = run_x2(oz, handle, "N", "N", Ai, Bi, 12)
    re, _ = exact_gemm("N", "N", Ai, Bi)
    assert all(Fraction(hi[i, j]) + Fraction(lo[i, j]) == re[i][j] for i in range(9) for j in range(7))


def test_x2_nonfinite_rows_and_arguments(oz, handle):
    rng = np.random.default_rng(8)
    m, n, k = 40, 30, 50
    A, B = wide(rng, (m, k), 5), wide(rng, (k, n), 5)
    A[3, 7] = np.nan
    B[11, 4] = np.inf
    st, rep, hi, lo = run_x2(oz, handle, "N", "N", A, B, 9)
    assert rep.status == oz.OZ_ERR_NONFINITE
    assert np.all(np.isnan(hi[3])) and np.all(np.isnan(lo[3])) and np.all(np.isnan(hi[:, 4]))
    Ac, Bc = A.copy(), B.copy()
    Ac[3] = 0.0
    Bc[:, 4] = 0.0
    whi, wlo = oracle.emu_gemm_x2("N", "N", Ac, Bc, 9)
    keep = np.ones((m, n), bool)
    keep[3] = False
    keep[:, 4] = False
    assert np.array_equal(hi[keep], whi[keep]) and np.array_equal(lo[keep], wlo[keep])
    dA, _ = to_dev(A)
    dB, _ = to_dev(B)
    dH, _ = to_dev(np.zeros((m, n)))
    assert oz.oz_dgemm_x2(handle, "N", "N", m, n, k, dA, m, dB, k, dH, None, m, oz.prec(7), check=False) == 12
    assert oz.oz_dgemm_x2(handle, "N", "N", m, n, k, dA, m, dB, k, dH, dH, m, oz.prec(7), check=False) == 12
    dL, _ = to_dev(np.zeros((m, n)))
    assert oz.oz_dgemm_x2(handle, "N", "N", m, n, k, dA, m, dB, k, dH, dL, m, oz.prec(0, tol=1e-10),
                          check=False) == 14


def test_x2_full_size_samples_and_error(oz, handle):
    rng = np.random.default_rng(21)
    n = 2048
    A = np.asfortranarray(rng.standard_normal((n, n)))
    B = np.asfortranarray(rng.standard_normal((n, n)))
    dA = torch.from_numpy(A.ravel(order="F")).cuda()
    dB = torch.from_numpy(B.ravel(order="F")).cuda()
    dH = torch.zeros(n * n, dtype=torch.float64, device="cuda")
    dL = torch.zeros(n * n, dtype=torch.float64, device="cuda")
    rows = np.sort(rng.choice(n, 6, replace=False))
    cols = np.sort(rng.choice(n, 6, replace=False))
    re, _ = exact_gemm("N", "N", A[rows], B[:, cols])
    scale = float(np.abs(A[rows]).max(1).max() * np.abs(B[:, cols]).max(0).max())
    errs = {}
    for s in (8, 11, 14):
        print("x2 full size s=%d" % s, flush=True)
        oz.oz_dgemm_x2(handle, "N", "N", n, n, n, dA, n, dB, n, dH, dL, n, oz.prec(s))
        torch.cuda.synchronize()
        hi = from_dev(dH, n, n, n)[np.ix_(rows, cols)]
        lo = from_dev(dL, n, n, n)[np.ix_(rows, cols)]
        whi, wlo = oracle.emu_gemm_x2("N", "N", A, B, s, rows=rows, cols=cols)
        assert np.array_equal(hi, whi) and np.array_equal(lo, wlo)
        errs[s] = max(abs(float(Fraction(hi[a, b]) + Fraction(lo[a, b]) - re[a][b])) for a in range(6)
                      for b in range(6)) / scale
    print("x2 errors vs exact:", {s: "%.2g" % e for s, e in errs.items()})
    assert errs[8] > 1e-18 and errs[11] < 1e-19 and errs[14] < 1e-24
