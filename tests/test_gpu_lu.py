"""LU-based complex inversion with emulated ZGEMM updates (oz_zgetrf /
oz_zgetri) against the oracle (oracle/lu.py): pivots, info, factors and
inverse bit-exact over ragged sizes, panel widths and split numbers; the
inverse from the oracle's own factors bit-exact too; a singular matrix;
argument errors; and at the benchmark's size (n = 4096) the properties that
hold at any size: pivot bounds, P A = L U and A X = I to the accuracy of s."""
import numpy as np
import pytest
import torch

from gpu_util import from_dev, to_dev
from oracle import lu

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


def cmat(rng, n):
    return np.asfortranarray(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))


def gpu_getrf(oz, handle, A, nb, s, pad=3):
    n = A.shape[0]
    dA, lda = to_dev(A, n + pad)
    ipiv = torch.full((max(n, 1),), -1, dtype=torch.int32, device="cuda")
    info = oz.oz_zgetrf(handle, n, dA, lda, ipiv, nb, oz.prec(s))
    torch.cuda.synchronize()
    return dA, lda, ipiv, info


def gpu_getri(oz, handle, dLU, lda, ipiv, n, nb, s, pad=5):
    dX, ldx = to_dev(np.zeros((n, n), complex, order="F"), n + pad)
    oz.oz_zgetri(handle, n, dLU, lda, ipiv, dX, ldx, nb, oz.prec(s))
    torch.cuda.synchronize()
    return from_dev(dX, n, n, ldx)


CASES = [(1, 16, 7), (5, 2, 7), (37, 16, 3), (64, 64, 7), (100, 32, 7), (130, 32, 5), (130, 64, 14),
         (200, 48, 9), (257, 64, 7), (300, 0, 7), (600, 0, 6), (520, 256, 7), (700, 200, 4)]


@pytest.mark.parametrize("n,nb,s", CASES)
def test_getrf_getri_bit_exact(oz, handle, n, nb, s):
    rng = np.random.default_rng(1000 + 7 * n + s)
    A = cmat(rng, n)
    dA, lda, ipiv, info = gpu_getrf(oz, handle, A, nb, s)
    LU_ref, piv_ref, info_ref = lu.getrf(A, nb or 128, s)
    print("n=%d nb=%d s=%d" % (n, nb, s), flush=True)
    assert info == info_ref == 0
    assert np.array_equal(ipiv.cpu().numpy(), piv_ref)
    LU = from_dev(dA, n, n, lda)
    assert np.array_equal(LU, LU_ref)
    X = gpu_getri(oz, handle, dA, lda, ipiv, n, nb, s)
    X_ref = lu.getri(LU_ref, piv_ref, nb or 256, s)
    assert np.array_equal(X, X_ref)


def test_getrf_bit_exact_tall_panels(oz, handle):
    # rows beyond 2048 below the first panels: the panel runs 4 rows per thread
    rng = np.random.default_rng(2100)
    n, nb, s = 2100, 32, 3
    A = cmat(rng, n)
    print("n=%d nb=%d s=%d" % (n, nb, s), flush=True)
    dA, lda, ipiv, info = gpu_getrf(oz, handle, A, nb, s, pad=1)
    LU_ref, piv_ref, info_ref = lu.getrf(A, nb, s)
    assert info == info_ref == 0
    assert np.array_equal(ipiv.cpu().numpy(), piv_ref)
    assert np.array_equal(from_dev(dA, n, n, lda), LU_ref)


def test_getrf_matches_lapack_pivots_beyond_4096_rows(oz, handle):
    # rows beyond 4096 (8 rows per thread in the panel): at s = 14 the updates
    # are FP64-accurate, so the pivots are LAPACK's (same rule) and the factors
    # reproduce P A to rounding
    import scipy.linalg
    rng = np.random.default_rng(5000)
    n, nb = 5000, 64
    A = cmat(rng, n)
    print("n=%d nb=%d s=14" % (n, nb), flush=True)
    dA, lda, ipiv, info = gpu_getrf(oz, handle, A, nb, 14, pad=0)
    assert info == 0
    lu_ref, piv_ref = scipy.linalg.lu_factor(A)
    assert np.array_equal(ipiv.cpu().numpy(), piv_ref)
    LU = from_dev(dA, n, n, lda)
    assert np.abs(LU - lu_ref).max() / np.abs(lu_ref).max() < 1e-11


@pytest.mark.parametrize("n,nb,s", [(100, 32, 5), (257, 64, 6), (300, 0, 7)])
def test_getrf_getri_balanced_bit_exact(oz, handle, n, nb, s):
    # balanced digits in every emulated product of the factorisation and solves
    rng = np.random.default_rng(5000 + n + s)
    A = cmat(rng, n)
    dA, lda = to_dev(A, n + 2)
    ipiv = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    p = oz.prec(s, digits=1)
    info = oz.oz_zgetrf(handle, n, dA, lda, ipiv, nb, p)
    torch.cuda.synchronize()
    LU_ref, piv_ref, info_ref = lu.getrf(A, nb or 128, s, balanced=True)
    assert info == info_ref == 0
    assert np.array_equal(ipiv.cpu().numpy(), piv_ref)
    assert np.array_equal(from_dev(dA, n, n, lda), LU_ref)
    dX, ldx = to_dev(np.zeros((n, n), complex, order="F"), n + 1)
    oz.oz_zgetri(handle, n, dA, lda, ipiv, dX, ldx, nb, p)
    torch.cuda.synchronize()
    assert np.array_equal(from_dev(dX, n, n, ldx), lu.getri(LU_ref, piv_ref, nb or 256, s, balanced=True))


def test_getrf_matches_lapack_pivots_beyond_8192_rows(oz, handle):
    # the first panel has more rows than the register panel holds (8192): it
    # runs the global-memory panel kernel; s = 14 as above
    import scipy.linalg
    rng = np.random.default_rng(8300)
    n, nb = 8300, 128
    A = cmat(rng, n)
    print("n=%d nb=%d s=14" % (n, nb), flush=True)
    dA, lda, ipiv, info = gpu_getrf(oz, handle, A, nb, 14, pad=0)
    assert info == 0
    lu_ref, piv_ref = scipy.linalg.lu_factor(A)
    assert np.array_equal(ipiv.cpu().numpy(), piv_ref)
    LU = from_dev(dA, n, n, lda)
    assert np.abs(LU - lu_ref).max() / np.abs(lu_ref).max() < 1e-11


def test_getri_from_oracle_factors(oz, handle):
    # the inverse step alone, fed the oracle's factors and pivots
    rng = np.random.default_rng(77)
    n, nb, s = 150, 40, 6
    LU_ref, piv_ref, _ = lu.getrf(cmat(rng, n), nb, s)
    dLU, lda = to_dev(LU_ref, n + 1)
    ipiv = torch.from_numpy(piv_ref.astype(np.int32)).cuda()
    X = gpu_getri(oz, handle, dLU, lda, ipiv, n, nb, s)
    assert np.array_equal(X, lu.getri(LU_ref, piv_ref, nb, s))


def test_wide_range_entries(oz, handle):
    # rows and columns spread over 2^-30 .. 2^30: the per-row / per-column
    # scales of each emulated update differ widely
    rng = np.random.default_rng(21)
    n, nb, s = 96, 32, 8
    A = cmat(rng, n) * np.exp2(rng.integers(-30, 31, n))[:, None] * np.exp2(rng.integers(-30, 31, n))[None, :]
    A = np.asfortranarray(A)
    dA, lda, ipiv, info = gpu_getrf(oz, handle, A, nb, s)
    LU_ref, piv_ref, _ = lu.getrf(A, nb, s)
    assert np.array_equal(ipiv.cpu().numpy(), piv_ref)
    assert np.array_equal(from_dev(dA, n, n, lda), LU_ref)
    assert np.array_equal(gpu_getri(oz, handle, dA, lda, ipiv, n, nb, s), lu.getri(LU_ref, piv_ref, nb, s))


def test_singular_info(oz, handle):
    rng = np.random.default_rng(5)
    n = 50
    A = cmat(rng, n)
    A[:, 23] = 0
    A[:, 40] = 0
    dA, lda, ipiv, info = gpu_getrf(oz, handle, A, 16, 7)
    LU_ref, piv_ref, info_ref = lu.getrf(A, 16, 7)
    assert info == info_ref == 24
    assert np.array_equal(ipiv.cpu().numpy(), piv_ref)
    assert np.array_equal(from_dev(dA, n, n, lda), LU_ref)


def test_closed_form_inverse(oz, handle):
    # permutation times a power-of-two diagonal: every step exact
    rng = np.random.default_rng(8)
    n = 70
    d = np.exp2(rng.integers(-40, 41, n)) * (1 - 1j * rng.integers(0, 2, n))
    A = np.asfortranarray(np.eye(n)[rng.permutation(n)] @ np.diag(d))
    dA, lda, ipiv, info = gpu_getrf(oz, handle, A, 16, 3)
    X = gpu_getri(oz, handle, dA, lda, ipiv, n, 16, 3)
    assert info == 0
    assert np.array_equal(X, np.diag(1 / d) @ A.T.real.astype(bool).astype(float))


def test_empty_and_argument_errors(oz, handle):
    t = torch.zeros(8, dtype=torch.float64, device="cuda")
    piv = torch.zeros(4, dtype=torch.int32, device="cuda")
    assert oz.oz_zgetrf(handle, 0, None, 1, None, 0, oz.prec(7)) == 0
    assert oz.oz_zgetri(handle, 0, None, 1, None, None, 1, 0, oz.prec(7)) == 0
    assert oz.oz_zgetrf(handle, -1, t, 1, piv, 0, oz.prec(7), check=False)[0] == 2
    assert oz.oz_zgetrf(handle, 2, t, 1, piv, 0, oz.prec(7), check=False)[0] == 4
    assert oz.oz_zgetrf(handle, 2, t, 2, piv, -1, oz.prec(7), check=False)[0] == 6
    assert oz.oz_zgetrf(handle, 2, None, 2, piv, 0, oz.prec(7), check=False)[0] == oz.OZ_ERR_ARG
    assert oz.oz_zgetri(handle, 2, t, 2, piv, t, 2, 0, oz.prec(7), check=False) == oz.OZ_ERR_ARG
    assert oz.oz_zgetri(handle, 2, t, 2, piv, t, 1, 0, oz.prec(7), check=False) == 7
    assert oz.oz_zgetri(handle, 2, t, 1, piv, t, 2, 0, oz.prec(7), check=False) == 4


def perm_order(piv):
    order = np.arange(len(piv))
    for j, p in enumerate(piv):
        order[[j, p]] = order[[p, j]]
    return order


# Bounds.  A random complex Gaussian matrix of order n has condition number of
# order n; an emulated product at s slices carries a relative error of about
# 2^(-7 s + 6) of its operand scales (1e-12 at s = 7), and at s = 14 sits at
# the FP64 floor.  So at s = 7 the factors reproduce A to about 1e-11 and the
# inverse is good to cond * 1e-12 ~ 4e-9 (bounds 1e-9, 1e-7); at s = 14 the
# inverse is as good as the native one (residual within 10x of its residual).
@pytest.mark.parametrize("s,bound_lu,bound_inv", [(7, 1e-9, 1e-7), (14, 1e-12, None)])
def test_full_size_properties(oz, handle, s, bound_lu, bound_inv):
    n, nb = 4096, 64
    g = torch.Generator(device="cpu").manual_seed(4096 + s)
    A = torch.complex(torch.randn(n, n, generator=g, dtype=torch.float64),
                      torch.randn(n, n, generator=g, dtype=torch.float64))
    dA = torch.view_as_real(A.T.contiguous()).reshape(-1).cuda()  # column-major interleaved
    ipiv = torch.empty(n, dtype=torch.int32, device="cuda")
    print("n=%d s=%d" % (n, s), flush=True)
    info = oz.oz_zgetrf(handle, n, dA, n, ipiv, nb, oz.prec(s))
    assert info == 0
    piv = ipiv.cpu().numpy()
    assert np.all(piv >= np.arange(n)) and np.all(piv < n)
    LUc = torch.view_as_complex(dA.view(n, n, 2)).T  # LU[i, j] (device, complex128)
    eye = torch.eye(n, dtype=torch.complex128, device="cuda")
    L = torch.tril(LUc, -1) + eye
    U = torch.triu(LUc)
    assert L.abs().max().item() <= np.sqrt(2) * (1 + 1e-12)
    Ad = A.cuda()
    PA = Ad[torch.from_numpy(perm_order(piv)).cuda()]
    err_lu = ((PA - L @ U).abs().max() / Ad.abs().max()).item()
    dX = torch.zeros(2 * n * n, dtype=torch.float64, device="cuda")
    oz.oz_zgetri(handle, n, dA, n, ipiv, dX, n, nb, oz.prec(s))
    X = torch.view_as_complex(dX.view(n, n, 2)).T
    resid = ((Ad @ X - eye).abs().max()).item()
    Xr = torch.linalg.inv(Ad)
    resid_native = ((Ad @ Xr - eye).abs().max()).item()
    err_inv = ((X - Xr).abs().max() / Xr.abs().max()).item()
    torch.cuda.synchronize()
    print("lu %.2e resid %.2e (native %.2e) inv %.2e" % (err_lu, resid, resid_native, err_inv), flush=True)
    assert err_lu < bound_lu
    if bound_inv is None:
        assert resid < 10 * resid_native
    else:
        assert err_inv < bound_inv


def test_tolerance_driven_products(oz, handle):
    # every emulated product of the factorisation and the solves picks its own
    # slice count for the tolerance (the starting rule, then growth until the
    # a-posteriori estimate passes): a tighter tolerance gives a smaller
    # residual, and at 1e-13 the inverse is as good as at fixed s = 14 to
    # within the condition number's amplification of 1e-13
    n = 1024
    rng = np.random.default_rng(1024)
    A = cmat(rng, n)
    Ad = torch.from_numpy(A).cuda()
    eye = torch.eye(n, dtype=torch.complex128, device="cuda")
    out = {}
    for tol in (1e-8, 1e-13):
        p = oz.prec(0, tol=tol)
        dA, lda = to_dev(A, n)
        ipiv = torch.empty(n, dtype=torch.int32, device="cuda")
        assert oz.oz_zgetrf(handle, n, dA, lda, ipiv, 0, p) == 0
        dX, ldx = to_dev(np.zeros((n, n), complex, order="F"), n)
        oz.oz_zgetri(handle, n, dA, lda, ipiv, dX, ldx, 0, p)
        X = torch.from_numpy(from_dev(dX, n, n, ldx)).cuda()
        out[tol] = float((Ad @ X - eye).abs().max())
    print("resid by tol", out, flush=True)
    assert out[1e-13] < out[1e-8] / 100
    assert out[1e-8] < 1e-8 * n * 10
    assert out[1e-13] < 1e-13 * n * 10

