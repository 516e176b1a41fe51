"""The BLAS offload layer on the GPU: dgemm_ / zgemm_ called with host
arrays (copied over PCIe) or device pointers (used in place), against the
oracle (bit-exact in the emulated modes) and the library's own calls."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import from_dev, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def blas():
    import paper_2503_22875_amd.blas as b
    torch.cuda.set_device(0)
    yield b
    b.oz_blas_set_mode("fp64_int8_7")


def wide(rng, shape, span, cplx=False):
    x = rng.standard_normal(shape)
    if cplx:
        x = x + 1j * rng.standard_normal(shape)
    return np.asfortranarray(x * np.exp2(rng.integers(-span, span + 1, size=shape)))


def padded(X, extra):
    """X stored with leading dimension rows + extra (a Fortran array)."""
    buf = np.zeros((X.shape[0] + extra, X.shape[1]), dtype=X.dtype, order="F")
    buf[:X.shape[0]] = X
    return buf


@pytest.mark.parametrize("s", [3, 7])
@pytest.mark.parametrize("ta,tb", [("N", "N"), ("T", "N"), ("N", "T"), ("T", "T")])
def test_dgemm_host_bit_exact(blas, s, ta, tb):
    rng = np.random.default_rng(s * 10 + ord(ta) + 2 * ord(tb))
    m, n, k = 130, 70, 257
    A = wide(rng, (m, k) if ta == "N" else (k, m), 20)
    B = wide(rng, (k, n) if tb == "N" else (n, k), 20)
    C0 = wide(rng, (m, n), 5)
    Ap, Bp, Cp = padded(A, 3), padded(B, 1), padded(C0, 2)
    assert blas.oz_blas_set_mode("fp64_int8_%d" % s)
    print("blas dgemm", s, ta, tb, flush=True)
    blas.dgemm_(ta, tb, m, n, k, -1.25, Ap, Ap.shape[0], Bp, Bp.shape[0], 0.5, Cp, Cp.shape[0])
    want = oracle.emu_gemm(ta, tb, A, B, s, alpha=-1.25, beta=0.5, C=C0)
    assert np.array_equal(Cp[:m], want)
    assert np.all(Cp[m:] == 0.0)  # rows past m of the padded C are not touched
    st = blas.oz_blas_stats()
    assert st.last_info == 0 and st.last_slices == s


@pytest.mark.parametrize("ta,tb", [("N", "N"), ("C", "N"), ("T", "C"), ("C", "T")])
def test_zgemm_host_bit_exact(blas, ta, tb):
    rng = np.random.default_rng(ord(ta) * 3 + ord(tb))
    m, n, k = 90, 65, 140
    A = wide(rng, (m, k) if ta == "N" else (k, m), 15, True)
    B = wide(rng, (k, n) if tb == "N" else (n, k), 15, True)
    C0 = wide(rng, (m, n), 3, True)
    Cp = padded(C0, 1)
    assert blas.oz_blas_set_mode("fp64_int8_6")
    print("blas zgemm", ta, tb, flush=True)
    blas.zgemm_(ta, tb, m, n, k, 0.75 - 0.5j, A, A.shape[0], B, B.shape[0], -1.0 + 0.25j, Cp, Cp.shape[0])
    want = oracle.emu_gemm(ta, tb, A, B, 6, alpha=0.75 - 0.5j, beta=-1.0 + 0.25j, C=C0)
    assert np.array_equal(Cp[:m], want)


@pytest.mark.parametrize("s", [4, 6])
def test_balanced_mode_bit_exact(blas, s):
    # OZ_COMPUTE_MODE fp64_int8_bal<s>: balanced digits in dgemm_ and zgemm_
    rng = np.random.default_rng(40 + s)
    m, n, k = 100, 60, 130
    A, B, C0 = wide(rng, (m, k), 12), wide(rng, (k, n), 12), wide(rng, (m, n), 4)
    Cp = padded(C0, 2)
    assert blas.oz_blas_set_mode("fp64_int8_bal%d" % s)
    print("blas balanced", s, flush=True)
    blas.dgemm_("N", "T", m, n, k, 1.5, A, m, np.asfortranarray(B.T), n, -0.5, Cp, Cp.shape[0])
    assert np.array_equal(Cp[:m], oracle.emu_gemm("N", "N", A, B, s, alpha=1.5, beta=-0.5, C=C0, balanced=True))
    assert blas.oz_blas_stats().mode == 3
    Az, Bz = wide(rng, (m, k), 8, True), wide(rng, (k, n), 8, True)
    Cz = np.zeros((m, n), complex, order="F")
    blas.zgemm_("N", "N", m, n, k, 1.0, Az, m, Bz, k, 0.0, Cz, m)
    assert np.array_equal(Cz, oracle.emu_gemm("N", "N", Az, Bz, s, balanced=True))


def test_device_pointers_used_in_place(blas):
    rng = np.random.default_rng(5)
    m, n, k = 100, 80, 120
    A, B = wide(rng, (m, k), 10), wide(rng, (k, n), 10)
    dA, lda = to_dev(A, m + 2)
    dB, ldb = to_dev(B)
    dC, ldc = to_dev(np.zeros((m, n)), m + 1)
    assert blas.oz_blas_set_mode("fp64_int8_7")
    before = blas.oz_blas_stats()
    print("blas device pointers", flush=True)
    blas.dgemm_("N", "N", m, n, k, 1.0, dA, lda, dB, ldb, 0.0, dC, ldc)
    after = blas.oz_blas_stats()
    assert after.bytes_to_device == before.bytes_to_device and after.bytes_to_host == before.bytes_to_host
    assert np.array_equal(from_dev(dC, m, n, ldc), oracle.emu_gemm("N", "N", A, B, 7))


def test_tolerance_mode_matches_the_library(blas):
    import paper_2503_22875_amd as oz
    rng = np.random.default_rng(9)
    m, n, k = 150, 120, 260
    A, B = wide(rng, (m, k), 30), wide(rng, (k, n), 30)
    C = np.zeros((m, n), order="F")
    assert blas.oz_blas_set_mode("fp64_int8_tol1e-11")
    print("blas tol", flush=True)
    blas.dgemm_("N", "N", m, n, k, 1.0, A, m, B, k, 0.0, C, m)
    s_used = blas.oz_blas_stats().last_slices
    h = oz.oz_create(0)
    try:
        dA, _ = to_dev(A)
        dB, _ = to_dev(B)
        dC, _ = to_dev(np.zeros((m, n)))
        st, rep = oz.oz_dgemm(h, "N", "N", m, n, k, 1.0, dA, m, dB, k, 0.0, dC, m, oz.prec(0, tol=1e-11, smax=12),
                              report=True)
        torch.cuda.synchronize()
        assert rep.slices_used == s_used
        assert np.array_equal(C, from_dev(dC, m, n, m))
    finally:
        oz.oz_destroy(h)
    ref = oracle.gemm_dd("N", "N", A, B)
    assert oracle.weighted_error(C, ref, np.abs(A).max(1), np.abs(B).max(0)) <= 2e-11


def test_beta_zero_does_not_read_c_and_alpha_zero_scales(blas):
    rng = np.random.default_rng(2)
    m, n, k = 40, 30, 50
    A, B = wide(rng, (m, k), 4), wide(rng, (k, n), 4)
    C = np.full((m, n), np.nan, order="F")
    assert blas.oz_blas_set_mode("fp64_int8_5")
    blas.dgemm_("N", "N", m, n, k, 2.0, A, m, B, k, 0.0, C, m)
    assert np.array_equal(C, oracle.emu_gemm("N", "N", A, B, 5, alpha=2.0))
    C2 = wide(rng, (m, n), 4)
    want = 3.0 * C2
    blas.dgemm_("N", "N", m, n, k, 0.0, A, m, B, k, 3.0, C2, m)  # C <- beta C on the GPU
    assert np.array_equal(C2, want)


def test_native_mode(blas):
    rng = np.random.default_rng(4)
    m, n, k = 200, 150, 300
    A = rng.standard_normal((m, k)) + 1j * rng.standard_normal((m, k))
    B = rng.standard_normal((k, n)) + 1j * rng.standard_normal((k, n))
    A, B = np.asfortranarray(A), np.asfortranarray(B)
    C = np.zeros((m, n), np.complex128, order="F")
    assert blas.oz_blas_set_mode("dgemm")
    print("blas native", flush=True)
    Bs = np.asfortranarray(B.conj().T)  # stored n x k; op = 'C' gives B back
    blas.zgemm_("N", "C", m, n, k, 1.0, A, m, Bs, n, 0.0, C, m)
    want = A @ B
    assert np.linalg.norm(C - want) / np.linalg.norm(want) < 1e-14
    assert blas.oz_blas_set_mode("fp64_int8_7")
