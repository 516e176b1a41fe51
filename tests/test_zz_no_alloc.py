"""GPU tests of the allocation-free entry point oz_gemm_noalloc: the same bits
as oz_dgemm / oz_zgemm (and the oracle) on two calls in a row, the second one
smaller (the fixed scratch keeps the first call's contents), for real and both
complex forms with both digit kinds; a call whose workspace exceeds the fixed
scratch is rejected without touching C; tolerance mode is rejected."""
import numpy as np
import pytest
import torch

import oracle
import paper_2503_22875_amd as oz
from gpu_util import from_dev, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def handle():
    torch.cuda.set_device(0)
    h = oz.oz_create(0)
    oz.oz_set_stream(h, torch.cuda.current_stream().cuda_stream)
    yield h
    oz.oz_destroy(h)


def _mat(rng, r, c, cplx, spread=8):
    X = rng.standard_normal((r, c)) * np.ldexp(1.0, rng.integers(-spread, spread + 1, size=(r, 1)))
    if cplx:
        X = X + 1j * rng.standard_normal((r, c)) * np.ldexp(1.0, rng.integers(-spread, spread + 1, size=(r, 1)))
    return np.asfortranarray(X)


def _run_pair(h, cplx, ta, tb, m, n, k, p, alpha, beta, seed):
    """C by oz_gemm_noalloc and by the allocating entry point, same inputs; also the oracle."""
    rng = np.random.default_rng(seed)
    A = _mat(rng, *((m, k) if ta == "N" else (k, m)), cplx)
    B = _mat(rng, *((k, n) if tb == "N" else (n, k)), cplx)
    C0 = _mat(rng, m, n, cplx)
    dA, lda = to_dev(A, A.shape[0] + 3)
    dB, ldb = to_dev(B, B.shape[0] + 1)
    dC1, ldc = to_dev(C0, m + 2)
    dC2, _ = to_dev(C0, m + 2)
    print("noalloc: cplx=%d %s%s m=%d n=%d k=%d s=%d zmode=%d digits=%d" %
          (cplx, ta, tb, m, n, k, p.slices, p.zmode, p.digits), flush=True)
    oz.oz_gemm_noalloc(h, cplx, ta, tb, m, n, k, alpha, dA, lda, dB, ldb, beta, dC1, ldc, p)
    fn = oz.oz_zgemm if cplx else oz.oz_dgemm
    fn(h, ta, tb, m, n, k, alpha, dA, lda, dB, ldb, beta, dC2, ldc, p)
    torch.cuda.synchronize()
    got = from_dev(dC1, m, n, ldc)
    ref = from_dev(dC2, m, n, ldc)
    bal = p.digits == 1
    if cplx and p.zmode == 3:
        want = oracle.emu_zgemm3(ta, tb, A, B, p.slices, alpha=alpha, beta=beta, C=C0, balanced=bal)
    else:
        want = oracle.emu_gemm(ta, tb, A, B, p.slices, alpha=alpha, beta=beta, C=C0, balanced=bal)
    # padding rows of the output buffer are untouched
    pad = dC1.cpu().numpy().reshape((m + 2, n), order="F")[m:]
    return got, ref, want, pad


CASES = [
    # (cplx, ta, tb, (m, n, k) first, (m, n, k) second, s, zmode, digits, alpha, beta)
    (0, "N", "T", (300, 250, 400), (70, 50, 33), 7, 0, 0, 1.5, -0.5),
    (0, "T", "N", (257, 129, 515), (1, 3, 2), 6, 0, 1, 1.0, 0.0),
    (1, "N", "N", (200, 180, 300), (40, 33, 17), 6, 4, 0, 1.0 - 0.5j, 0.25j),
    (1, "C", "T", (150, 190, 260), (31, 9, 70), 7, 4, 1, 1.0, 0.0),
    (1, "N", "C", (260, 200, 310), (65, 64, 63), 6, 3, 1, 1.0, 0.0),
    (1, "T", "N", (199, 201, 129), (17, 19, 23), 5, 3, 0, -2.0, 1.0 + 1.0j),
]


@pytest.mark.parametrize("cplx,ta,tb,big,small,s,zmode,digits,alpha,beta", CASES)
def test_noalloc_matches_entry_point_twice(handle, cplx, ta, tb, big, small, s, zmode, digits, alpha, beta):
    p = oz.prec(s, zmode=zmode, digits=digits)
    for seed, (m, n, k) in enumerate((big, small)):
        got, ref, want, pad = _run_pair(handle, cplx, ta, tb, m, n, k, p, alpha, beta, seed)
        assert np.array_equal(got, ref), (m, n, k)
        assert np.array_equal(got, want), (m, n, k)
        assert np.all(pad == 0)


def test_noalloc_rejects_beyond_scratch(handle):
    # DGEMM 4096^3 at s = 7 needs 7 * 4096 * 4096 bytes of slices per operand, beyond 64 MiB
    n = 4096
    p = oz.prec(7)
    need = oz.oz_workspace_size(handle, "N", "N", n, n, n, 0, p)
    assert need > oz.OZ_NOALLOC_SCRATCH_BYTES
    A = torch.ones(n * n, dtype=torch.float64, device="cuda")
    B = torch.ones(n * n, dtype=torch.float64, device="cuda")
    C = torch.full((n * n,), 3.0, dtype=torch.float64, device="cuda")
    st = oz.oz_gemm_noalloc(handle, 0, "N", "N", n, n, n, 1.0, A, n, B, n, 0.0, C, n, p, check=False)
    torch.cuda.synchronize()
    assert st == oz.OZ_ERR_ALLOC
    assert bool(torch.all(C == 3.0))


def test_noalloc_argument_errors(handle):
    A = torch.zeros(64, dtype=torch.float64, device="cuda")
    assert oz.oz_gemm_noalloc(handle, 0, "N", "N", 8, 8, 8, 1.0, A, 8, A, 8, 0.0, A, 8,
                              oz.prec(0, tol=1e-10), check=False) == 14
    assert oz.oz_gemm_noalloc(handle, 2, "N", "N", 8, 8, 8, 1.0, A, 8, A, 8, 0.0, A, 8, oz.prec(6),
                              check=False) == oz.OZ_ERR_ARG
    assert oz.oz_gemm_noalloc(handle, 0, "X", "N", 8, 8, 8, 1.0, A, 8, A, 8, 0.0, A, 8, oz.prec(6),
                              check=False) == 1
    assert oz.oz_gemm_noalloc(handle, 0, "N", "N", 8, 8, 8, 1.0, A, 4, A, 8, 0.0, A, 8, oz.prec(6),
                              check=False) == 8
    # quick return: m = 0 does nothing
    assert oz.oz_gemm_noalloc(handle, 1, "N", "N", 0, 8, 8, 1.0, A, 1, A, 8, 0.0, A, 1, oz.prec(6),
                              check=False) == 0
