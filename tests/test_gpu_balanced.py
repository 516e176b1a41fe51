"""Balanced (round-to-nearest) digits on the GPU (oz_prec_t.digits = 1)
against the oracle's emu_gemm(balanced=True): bit-exact over real and complex
products, every trans combination, padded leading dimensions, alpha/beta,
s = 1..8, every GEMM kernel shape, forced INT32 chunks and non-finite rows; at
full size (ZGEMM n = 4096, s = 7) sampled entries bit-exact and the error
below that of truncated digits at the same s; and the calls that do not take
balanced digits rejected."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import from_dev, to_dev

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
    x = rng.standard_normal(shape) * np.exp2(rng.integers(-span, span + 1, size=shape))
    if cplx:
        x = x + 1j * rng.standard_normal(shape) * np.exp2(rng.integers(-span, span + 1, size=shape))
    return np.asfortranarray(x)


def stored(rng, trans, rows, cols, span, cplx):
    return wide(rng, (cols, rows) if trans != "N" else (rows, cols), span, cplx)


def run(oz, handle, ta, tb, A, B, s, alpha=1.0, beta=0.0, C=None, kernel=0, kchunk=0, check=True):
    cplx = np.iscomplexobj(A)
    m = A.shape[0] if ta == "N" else A.shape[1]
    k = A.shape[1] if ta == "N" else A.shape[0]
    n = B.shape[1] if tb == "N" else B.shape[0]
    dA, lda = to_dev(A, A.shape[0] + 1)
    dB, ldb = to_dev(B, B.shape[0] + 2)
    C0 = np.zeros((m, n), A.dtype, order="F") if C is None else C
    dC, ldc = to_dev(C0, m + 3)
    fn = oz.oz_zgemm if cplx else oz.oz_dgemm
    st = fn(handle, ta, tb, m, n, k, alpha, dA, lda, dB, ldb, beta, dC, ldc,
            oz.prec(s, kernel=kernel, kchunk=kchunk, digits=1), check=check)
    torch.cuda.synchronize()
    return st, from_dev(dC, m, n, ldc)


TRANS_R = [("N", "N"), ("T", "N"), ("N", "T"), ("T", "T")]
TRANS_Z = [("N", "N"), ("C", "N"), ("N", "C"), ("T", "C"), ("C", "T")]


@pytest.mark.parametrize("s", [1, 2, 3, 4, 5, 6, 7, 8])
@pytest.mark.parametrize("ta,tb", TRANS_R)
def test_dgemm_balanced_bit_exact(oz, handle, s, ta, tb):
    rng = np.random.default_rng(100 * s + ord(ta) + 3 * ord(tb))
    m, n, k = 131, 77, 150
    A = stored(rng, ta, m, k, 12, False)
    B = stored(rng, tb, k, n, 12, False)
    C = wide(rng, (m, n), 4)
    _, got = run(oz, handle, ta, tb, A, B, s, alpha=-1.5, beta=0.75, C=C)
    ref = oracle.emu_gemm(ta, tb, A, B, s, alpha=-1.5, beta=0.75, C=C, balanced=True)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("s", [1, 3, 6, 7, 8])
@pytest.mark.parametrize("ta,tb", TRANS_Z)
def test_zgemm_balanced_bit_exact(oz, handle, s, ta, tb):
    rng = np.random.default_rng(1000 + 10 * s + ord(ta) + 7 * ord(tb))
    m, n, k = 70, 45, 96
    A = stored(rng, ta, m, k, 10, True)
    B = stored(rng, tb, k, n, 10, True)
    C = wide(rng, (m, n), 3, True)
    al, be = complex(0.5, -2.0), complex(-1.0, 0.25)
    _, got = run(oz, handle, ta, tb, A, B, s, alpha=al, beta=be, C=C)
    ref = oracle.emu_gemm(ta, tb, A, B, s, alpha=al, beta=be, C=C, balanced=True)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("kernel", [1, 2, 3])
@pytest.mark.parametrize("cplx", [False, True])
def test_balanced_every_kernel_shape(oz, handle, kernel, cplx):
    rng = np.random.default_rng(7 + kernel + 10 * cplx)
    A = wide(rng, (200, 130), 8, cplx)
    B = wide(rng, (130, 150), 8, cplx)
    for s in (2, 7, 8):
        _, got = run(oz, handle, "N", "N", A, B, s, kernel=kernel)
        assert np.array_equal(got, oracle.emu_gemm("N", "N", A, B, s, balanced=True)), s


@pytest.mark.parametrize("cplx", [False, True])
def test_balanced_forced_chunks(oz, handle, cplx):
    rng = np.random.default_rng(31 + cplx)
    A = wide(rng, (90, 700), 6, cplx)
    B = wide(rng, (700, 60), 6, cplx)
    for s, kc in ((4, 128), (7, 64), (8, 256)):
        _, got = run(oz, handle, "N", "N", A, B, s, kchunk=kc)
        assert np.array_equal(got, oracle.emu_gemm("N", "N", A, B, s, kc=kc, balanced=True)), (s, kc)


def test_balanced_digit_edge_values(oz, handle):
    # ties (x 2^(6-E+8(s-1)) = integer + 1/2), digits at -128, subnormals,
    # zeros and the row maximum itself, at s = 1, 2 and 8
    rng = np.random.default_rng(5)
    m, n, k = 40, 33, 64
    A = wide(rng, (m, k), 3)
    A[0, :8] = [1.5, 2.0 ** -6, -(2.0 ** -6), 3 * 2.0 ** -7, 0.0, -0.0, 2.0 ** -1070, -(2.0 ** -1074)]
    A[1, :4] = [1.0, -(0.5 + 2.0 ** -9), 0.5 + 2.0 ** -8, -(2.0 ** -8)]
    A[2, :] = -np.abs(A[2, :])
    B = wide(rng, (k, n), 3)
    B[:, 0] = 2.0 ** -1060 * rng.standard_normal(k)
    for s in (1, 2, 8):
        _, got = run(oz, handle, "N", "N", A, B, s)
        assert np.array_equal(got, oracle.emu_gemm("N", "N", A, B, s, balanced=True)), s


@pytest.mark.parametrize("cplx", [False, True])
def test_balanced_nonfinite_rows(oz, handle, cplx):
    rng = np.random.default_rng(9 + cplx)
    m, n, k = 50, 40, 48
    A, B = wide(rng, (m, k), 4, cplx), wide(rng, (k, n), 4, cplx)
    A[3, 7] = np.inf
    B[9, 5] = np.nan
    _, got = run(oz, handle, "N", "N", A, B, 6)
    bad = np.zeros((m, n), bool)
    bad[3, :] = True
    bad[:, 5] = True
    assert np.all(np.isnan(got[bad]))
    A2, B2 = A.copy(), B.copy()
    A2[3, :] = 0
    B2[:, 5] = 0
    ref = oracle.emu_gemm("N", "N", A2, B2, 6, balanced=True)
    assert np.array_equal(got[~bad], ref[~bad])


def test_balanced_rejections(oz, handle):
    d = torch.zeros(64, dtype=torch.float64, device="cuda")
    z = torch.zeros(128, dtype=torch.float64, device="cuda")

    def dg(p):
        return oz.oz_dgemm(handle, "N", "N", 4, 4, 4, 1.0, d, 4, d, 4, 0.0, d, 4, p, check=False)

    assert dg(oz.prec(9, digits=1)) == 14
    assert dg(oz.prec(0, tol=1e-10, digits=1)) == 0  # tolerance-driven calls take balanced digits
    assert dg(oz.prec(7, digits=2)) == 14
    assert dg(oz.prec(7, digits=1, kchunk=18752)) == 14  # beyond s * kc * 128^2 <= 2^31 - 1
    assert dg(oz.prec(7, digits=1, kchunk=18688)) == 0
    lo = torch.zeros(64, dtype=torch.float64, device="cuda")
    assert oz.oz_dgemm_x2(handle, "N", "N", 4, 4, 4, d, 4, d, 4, d, lo, 4, oz.prec(7, digits=1), check=False) == 14


def test_balanced_full_size_zgemm(oz, handle):
    # ZGEMM n = 4096, s = 7: sampled entries bit-exact; error against the native
    # product below that of truncated digits at the same s
    import workloads
    n, s = 4096, 7
    A, B = workloads.zgemm_rowexp(n, seed=0)
    dA, _ = to_dev(A)
    dB, _ = to_dev(B)
    dC, _ = to_dev(np.zeros((n, n), complex, order="F"))
    dT, _ = to_dev(np.zeros((n, n), complex, order="F"))
    print("zgemm n=%d s=%d balanced" % (n, s), flush=True)
    oz.oz_zgemm(handle, "N", "N", n, n, n, 1.0, dA, n, dB, n, 0.0, dC, n, oz.prec(s, digits=1, zmode=4))
    oz.oz_zgemm(handle, "N", "N", n, n, n, 1.0, dA, n, dB, n, 0.0, dT, n, oz.prec(s, zmode=4))
    torch.cuda.synchronize()
    rng = np.random.default_rng(0)
    rows = np.sort(rng.choice(n, 24, replace=False))
    cols = np.sort(rng.choice(n, 20, replace=False))
    C = from_dev(dC, n, n, n)
    ref = oracle.emu_gemm("N", "N", A, B, s, rows=rows, cols=cols, balanced=True)
    assert np.array_equal(C[np.ix_(rows, cols)], ref)
    Ad = torch.from_numpy(A).cuda()
    Bd = torch.from_numpy(B).cuda()
    N = (Ad @ Bd).cpu().numpy()
    T = from_dev(dT, n, n, n)
    eb = np.linalg.norm(C - N) / np.linalg.norm(N)
    et = np.linalg.norm(T - N) / np.linalg.norm(N)
    print("err balanced %.3e truncated %.3e" % (eb, et), flush=True)
    assert eb < et / 4


@pytest.mark.parametrize("s", [3, 6, 7, 8])
@pytest.mark.parametrize("ta,tb", [("N", "N"), ("C", "N"), ("T", "C")])
def test_zgemm_3m_balanced_bit_exact(oz, handle, s, ta, tb):
    rng = np.random.default_rng(3000 + 10 * s + ord(ta) + 7 * ord(tb))
    m, n, k = 66, 50, 90
    A = stored(rng, ta, m, k, 10, True)
    B = stored(rng, tb, k, n, 10, True)
    C = wide(rng, (m, n), 3, True)
    al, be = complex(1.5, 0.5), complex(0.0, -1.0)
    dA, lda = to_dev(A, A.shape[0] + 1)
    dB, ldb = to_dev(B, B.shape[0] + 2)
    dC, ldc = to_dev(C, m + 3)
    oz.oz_zgemm(handle, ta, tb, m, n, k, al, dA, lda, dB, ldb, be, dC, ldc, oz.prec(s, zmode=3, digits=1))
    torch.cuda.synchronize()
    got = from_dev(dC, m, n, ldc)
    ref = oracle.emu_zgemm3(ta, tb, A, B, s, alpha=al, beta=be, C=C, balanced=True)
    assert np.array_equal(got, ref)


def test_zgemm_3m_balanced_full_size(oz, handle):
    # the benchmark's form (3M) at n = 4096, s = 7 with balanced digits:
    # sampled entries bit-exact, error far below the truncated form's
    import workloads
    n, s = 4096, 7
    A, B = workloads.zgemm_rowexp(n, seed=0)
    dA, _ = to_dev(A)
    dB, _ = to_dev(B)
    dC, _ = to_dev(np.zeros((n, n), complex, order="F"))
    print("zgemm 3M n=%d s=%d balanced" % (n, s), flush=True)
    oz.oz_zgemm(handle, "N", "N", n, n, n, 1.0, dA, n, dB, n, 0.0, dC, n, oz.prec(s, zmode=3, digits=1))
    torch.cuda.synchronize()
    rng = np.random.default_rng(1)
    rows = np.sort(rng.choice(n, 16, replace=False))
    cols = np.sort(rng.choice(n, 16, replace=False))
    C = from_dev(dC, n, n, n)
    ref = oracle.emu_zgemm3("N", "N", A, B, s, rows=rows, cols=cols, balanced=True)
    assert np.array_equal(C[np.ix_(rows, cols)], ref)
    N = (torch.from_numpy(A).cuda() @ torch.from_numpy(B).cuda()).cpu().numpy()
    err = np.linalg.norm(C - N) / np.linalg.norm(N)
    print("err 3M balanced %.3e" % err, flush=True)
    assert err < 3e-14


def run_tol_bal(oz, handle, A, B, tol, sstart=0):
    cplx = np.iscomplexobj(A)
    m, k = A.shape
    n = B.shape[1]
    dA, lda = to_dev(A)
    dB, ldb = to_dev(B)
    dC, ldc = to_dev(np.zeros((m, n), A.dtype, order="F"))
    fn = oz.oz_zgemm if cplx else oz.oz_dgemm
    st, rep = fn(handle, "N", "N", m, n, k, 1.0, dA, lda, dB, ldb, 0.0, dC, ldc,
                 oz.prec(0, tol=tol, sstart=sstart, digits=1), report=True)
    torch.cuda.synchronize()
    return from_dev(dC, m, n, ldc), rep


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("tol", [1e-6, 1e-10, 1e-13])
def test_balanced_tolerance_mode(oz, handle, cplx, tol):
    # the result is the fresh balanced product at the final s (chunks of the
    # smax = 8 plan), and the tolerance is met
    rng = np.random.default_rng(60 + cplx + int(-np.log10(tol)))
    A, B = wide(rng, (150, 200), 6, cplx), wide(rng, (200, 120), 6, cplx)
    got, rep = run_tol_bal(oz, handle, A, B, tol)
    s = rep.slices_used
    print("balanced tol %g: s %d, fallbacks %d, resid %.3g" % (tol, s, rep.fallbacks, rep.resid_est), flush=True)
    assert 1 <= s <= 8
    want = oracle.emu_gemm("N", "N", A, B, s, kc=oracle.kchunk(8, cplx, balanced=True), balanced=True)
    assert np.array_equal(got, want)
    ref = oracle.gemm_dd("N", "N", A, B)
    wa = np.maximum(np.abs(A.real), np.abs(A.imag)).max(1)
    wb = np.maximum(np.abs(B.real), np.abs(B.imag)).max(0)
    # the check stops at half the tolerance, so the true error is within it
    assert oracle.weighted_error(got, ref, wa, wb) <= tol
    if s < 8:
        assert rep.resid_est <= tol / 2


def test_balanced_tolerance_growth_from_a_low_start(oz, handle):
    # each growth step splits again and recomputes: the result is the fresh
    # balanced product at the final s, not an incremental sum
    rng = np.random.default_rng(71)
    A, B = wide(rng, (100, 160), 4, True), wide(rng, (160, 90), 4, True)
    got, rep = run_tol_bal(oz, handle, A, B, 1e-12, sstart=2)
    assert rep.fallbacks >= 3 and rep.slices_used == 2 + rep.fallbacks
    want = oracle.emu_gemm("N", "N", A, B, rep.slices_used, kc=oracle.kchunk(8, True, balanced=True),
                           balanced=True)
    assert np.array_equal(got, want)

