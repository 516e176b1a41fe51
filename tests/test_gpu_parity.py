"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Bar: exponents, INT8 digits and INT32 anti-diagonal sums bit-exact; the FP64
result bit-exact as well, since both sides take the same FP64 operations in
the same order (the oracle's header states it).  Inputs are seeded; sizes span
several 64 x 64 tiles with ragged tails.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads
from gpu_util import complex_row_index, decode_slices, from_dev, stored_shape, to_dev

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


def wide(rng, shape, span=30, cplx=False):
    x = rng.standard_normal(shape) * np.exp2(rng.integers(-span, span + 1, size=shape))
    if cplx:
        x = x + 1j * rng.standard_normal(shape) * np.exp2(rng.integers(-span, span + 1, size=shape))
    return np.asfortranarray(x)


def with_specials(X, side, trans):
    """Put a zero vector, a subnormal-only vector and signed zeros into X."""
    X = X.copy(order="F")
    vec_is_row = (side == "A") == (trans.upper() == "N")
    if vec_is_row:
        if X.shape[0] > 2:
            X[0, :] = 0
            X[1, :] = X[1, :] * 2.0 ** -1060
    else:
        if X.shape[1] > 2:
            X[:, 0] = 0
            X[:, 1] = X[:, 1] * 2.0 ** -1060
    X.flat[-1] = -0.0
    return X


# ----------------------------------------------------------------- split (a1, a2)

SPLIT_CASES = [(side, trans, cplx) for side in "AB" for trans in "NTC" for cplx in (0, 1) if not (trans == "C" and not cplx)]


@pytest.mark.parametrize("side,trans,cplx", SPLIT_CASES)
@pytest.mark.parametrize("nv,k", [(1, 1), (63, 65), (130, 97)])
@pytest.mark.parametrize("s", [1, 7, 13])
def test_split_bit_exact(oz, handle, side, trans, cplx, nv, k, s):
    rng = np.random.default_rng(nv * 1000 + k + s)
    X = with_specials(wide(rng, stored_shape(side, trans, nv, k), 40, bool(cplx)), side, trans)
    E_ref, dig_ref = oracle.split(side, trans, X, s)
    rows_pad, kpad, nbytes = oz.oz_split_layout(side, cplx, nv, k, s)
    dX, ld = to_dev(X, X.shape[0] + 3)
    dE = torch.full((nv,), 12345, dtype=torch.int32, device="cuda")
    dS = torch.full((nbytes,), 99, dtype=torch.int8, device="cuda")
    print("split", side, trans, cplx, nv, k, s, flush=True)
    oz.oz_split(handle, side, trans, cplx, nv, k, dX, ld, s, dE, dS)
    torch.cuda.synchronize()
    assert np.array_equal(dE.cpu().numpy(), E_ref)
    dig = decode_slices(dS.cpu().numpy(), s, rows_pad, kpad)
    if not cplx:
        want = np.zeros((s, rows_pad, kpad), np.int8)
        want[:, :nv, :k] = dig_ref
    elif side == "B":
        want = np.zeros((s, rows_pad, kpad), np.int8)
        want[:, :nv, :2 * k] = dig_ref.reshape(s, nv, 2 * k)
    else:
        want = np.zeros((s, rows_pad, kpad), np.int8)
        r = complex_row_index(np.arange(nv))
        re, im = dig_ref[..., 0], dig_ref[..., 1]
        want[:, r, 0:2 * k:2] = re
        want[:, r, 1:2 * k:2] = -im
        want[:, r + 8, 0:2 * k:2] = im
        want[:, r + 8, 1:2 * k:2] = re
    assert np.array_equal(dig, want)


# ----------------------------------------------------------------- INT32 diagonals (a3)


@pytest.mark.parametrize("kernel", [1, 2, 3])
@pytest.mark.parametrize("cplx", [0, 1])
@pytest.mark.parametrize("m,n,k,s,kc", [(70, 65, 300, 7, 64), (64, 64, 128, 8, None), (130, 20, 33, 3, 128),
                                        (5, 7, 2000, 5, 512)])
def test_diagonal_sums_bit_exact(oz, handle, cplx, m, n, k, s, kc, kernel):
    rng = np.random.default_rng(m + n + k + s)
    A = wide(rng, (m, k), 20, bool(cplx))
    B = wide(rng, (k, n), 20, bool(cplx))
    kc = oracle.kchunk(s) if kc is None else kc
    ra, kpad, nba = oz.oz_split_layout("A", cplx, m, k, s)
    rb, _, nbb = oz.oz_split_layout("B", cplx, n, k, s)
    dA, lda = to_dev(A)
    dB, ldb = to_dev(B)
    sa = torch.zeros(nba, dtype=torch.int8, device="cuda")
    sb = torch.zeros(nbb, dtype=torch.int8, device="cuda")
    ea = torch.zeros(m, dtype=torch.int32, device="cuda")
    fb = torch.zeros(n, dtype=torch.int32, device="cuda")
    oz.oz_split(handle, "A", "N", cplx, m, k, dA, lda, s, ea, sa)
    oz.oz_split(handle, "B", "N", cplx, n, k, dB, ldb, s, fb, sb)
    nch = -(-kpad // kc)
    out = torch.full((nch * s * rb * ra,), -7, dtype=torch.int32, device="cuda")
    print("diag", cplx, m, n, k, s, kc, kernel, flush=True)
    oz.oz_diag_sums(handle, s, kc, ra, rb, kpad, sa, sb, out, kernel=kernel)
    torch.cuda.synchronize()
    got = out.cpu().numpy().reshape(nch, s, rb, ra).transpose(0, 1, 3, 2)  # [c, d-2, i, j]
    _, digA = oracle.split("A", "N", A, s)
    _, digB = oracle.split("B", "N", B, s)
    ref = oracle.diag_sums(digA, digB, s, kc=kc)
    if not cplx:
        assert ref.shape[0] == nch
        assert np.array_equal(got[:, :, :m, :n], ref)
        assert np.all(got[:, :, m:, :] == 0) and np.all(got[:, :, :, n:] == 0)
    else:
        Sr, Si = ref
        assert Sr.shape[0] == nch
        r = complex_row_index(np.arange(m))
        assert np.array_equal(got[:, :, r, :n], Sr)
        assert np.array_equal(got[:, :, r + 8, :n], Si)
    assert np.abs(got).max() <= 2 ** 31 - 1


# ----------------------------------------------------------------- FP64 result (a4, a5)


def run_gemm(oz, handle, cplx, ta, tb, A, B, s, alpha=1.0, beta=0.0, C0=None, kc=0, pad=0, kernel=0, zmode=0):
    m = A.shape[0] if ta == "N" else A.shape[1]
    k = A.shape[1] if ta == "N" else A.shape[0]
    n = B.shape[1] if tb == "N" else B.shape[0]
    dA, lda = to_dev(A, A.shape[0] + pad)
    dB, ldb = to_dev(B, B.shape[0] + pad)
    dt = np.complex128 if cplx else np.float64
    C0 = np.zeros((m, n), dt, order="F") if C0 is None else C0
    dC, ldc = to_dev(C0, m + pad)
    fn = oz.oz_zgemm if cplx else oz.oz_dgemm
    fn(handle, ta, tb, m, n, k, alpha, dA, lda, dB, ldb, beta, dC, ldc,
       oz.prec(s, kchunk=kc, kernel=kernel, zmode=zmode))
    torch.cuda.synchronize()
    return from_dev(dC, m, n, ldc)


GEMM_SHAPES = [(1, 1, 1), (63, 65, 33), (130, 70, 257), (64, 192, 64)]


@pytest.mark.parametrize("kernel", [0, 1, 2, 3, 4, 5])
@pytest.mark.parametrize("ta,tb", [("N", "N"), ("T", "N"), ("N", "T"), ("T", "T")])
@pytest.mark.parametrize("m,n,k", GEMM_SHAPES)
@pytest.mark.parametrize("s", [1, 3, 7, 8])
def test_dgemm_bit_exact(oz, handle, ta, tb, m, n, k, s, kernel):
    rng = np.random.default_rng(7 * m + 11 * n + 13 * k + s)
    A = wide(rng, (m, k) if ta == "N" else (k, m), 25)
    B = wide(rng, (k, n) if tb == "N" else (n, k), 25)
    print("dgemm", ta, tb, m, n, k, s, kernel, flush=True)
    got = run_gemm(oz, handle, 0, ta, tb, A, B, s, pad=2, kernel=kernel)
    assert np.array_equal(got, oracle.emu_gemm(ta, tb, A, B, s))


@pytest.mark.parametrize("kernel", [0, 1, 2, 3, 4, 5])
@pytest.mark.parametrize("ta,tb", [("N", "N"), ("C", "N"), ("T", "C"), ("C", "T")])
@pytest.mark.parametrize("m,n,k", GEMM_SHAPES)
@pytest.mark.parametrize("s", [2, 6, 7, 8])
def test_zgemm_bit_exact(oz, handle, ta, tb, m, n, k, s, kernel):
    rng = np.random.default_rng(17 * m + 19 * n + 23 * k + s)
    A = wide(rng, (m, k) if ta == "N" else (k, m), 25, True)
    B = wide(rng, (k, n) if tb == "N" else (n, k), 25, True)
    print("zgemm", ta, tb, m, n, k, s, kernel, flush=True)
    got = run_gemm(oz, handle, 1, ta, tb, A, B, s, pad=1, kernel=kernel)
    assert np.array_equal(got, oracle.emu_gemm(ta, tb, A, B, s))


@pytest.mark.parametrize("cplx", [0, 1])
@pytest.mark.parametrize("alpha,beta", [(1.0, 1.0), (-1.5, 0.25), (0.3 - 2j, 1.25 + 0.5j), (2.0, 0.0)])
def test_alpha_beta_bit_exact(oz, handle, cplx, alpha, beta):
    if not cplx and (isinstance(alpha, complex) or isinstance(beta, complex)):
        pytest.skip("complex scalars for zgemm only")
    rng = np.random.default_rng(3)
    m, n, k = 97, 70, 130
    A, B = wide(rng, (m, k), 10, bool(cplx)), wide(rng, (k, n), 10, bool(cplx))
    C0 = wide(rng, (m, n), 10, bool(cplx))
    got = run_gemm(oz, handle, cplx, "N", "N", A, B, 7, alpha, beta, C0)
    assert np.array_equal(got, oracle.emu_gemm("N", "N", A, B, 7, alpha=alpha, beta=beta, C=C0))


@pytest.mark.parametrize("kernel", [1, 2, 3])
@pytest.mark.parametrize("cplx", [0, 1])
@pytest.mark.parametrize("kc", [64, 128, 1024])
def test_forced_split_k_bit_exact(oz, handle, cplx, kc, kernel):
    rng = np.random.default_rng(kc)
    m, n, k = 70, 66, 1100
    A, B = wide(rng, (m, k), 10, bool(cplx)), wide(rng, (k, n), 10, bool(cplx))
    got = run_gemm(oz, handle, cplx, "N", "N", A, B, 7, kc=kc, kernel=kernel)
    assert np.array_equal(got, oracle.emu_gemm("N", "N", A, B, 7, kc=kc))


def test_config1_dgemm_parity_and_accuracy(oz, handle):
    A, B = workloads.dgemm_uniform(256, 256, 256, seed=0)
    got = run_gemm(oz, handle, 0, "N", "N", A, B, 7)
    assert np.array_equal(got, oracle.emu_gemm("N", "N", A, B, 7))
    ref = oracle.gemm_dd("N", "N", A, B)
    err = oracle.weighted_error(got, ref, np.abs(A).max(1), np.abs(B).max(0))
    print("config1 s=7 rel err %.3g" % err)
    assert err <= 1e-12


# ----------------------------------------------------------------- edge cases


def test_quick_returns(oz, handle):
    rng = np.random.default_rng(0)
    A, B, C0 = wide(rng, (5, 4), 3), wide(rng, (4, 6), 3), wide(rng, (5, 6), 3)
    # alpha = 0: C = beta*C
    assert np.array_equal(run_gemm(oz, handle, 0, "N", "N", A, B, 7, 0.0, 0.5, C0), 0.5 * C0)
    # alpha = 0, beta = 0: exact zeros even over NaN
    Cn = np.full((5, 6), np.nan)
    got = run_gemm(oz, handle, 0, "N", "N", A, B, 7, 0.0, 0.0, Cn)
    assert np.all(got == 0)
    # k = 0
    A0, B0 = np.zeros((5, 0), order="F"), np.zeros((0, 6), order="F")
    dA = torch.zeros(1, dtype=torch.float64, device="cuda")
    dC, ldc = to_dev(C0)
    oz.oz_dgemm(handle, "N", "N", 5, 6, 0, 1.0, dA, 5, dA, 1, 2.0, dC, ldc, oz.prec(7))
    torch.cuda.synchronize()
    assert np.array_equal(from_dev(dC, 5, 6, ldc), 2.0 * C0)
    # beta = 1 with alpha = 0: untouched; m = 0 / n = 0: nothing
    assert np.array_equal(run_gemm(oz, handle, 0, "N", "N", A, B, 7, 0.0, 1.0, C0), C0)
    oz.oz_dgemm(handle, "N", "N", 0, 6, 4, 1.0, dA, 1, dA, 4, 0.0, dC, 1, oz.prec(7))
    del A0, B0


def test_argument_errors_positions(oz, handle):
    d = torch.zeros(64, dtype=torch.float64, device="cuda")
    cases = [(("X", "N", 4, 4, 4, 4, 4, 4), 1), (("N", "X", 4, 4, 4, 4, 4, 4), 2), (("N", "N", -1, 4, 4, 4, 4, 4), 3),
             (("N", "N", 4, -1, 4, 4, 4, 4), 4), (("N", "N", 4, 4, -1, 4, 4, 4), 5), (("N", "N", 4, 4, 4, 3, 4, 4), 8),
             (("N", "N", 4, 4, 4, 4, 3, 4), 10), (("N", "N", 4, 4, 4, 4, 4, 3), 13), (("T", "N", 4, 4, 5, 4, 5, 4), 8)]
    for (ta, tb, m, n, k, lda, ldb, ldc), pos in cases:
        st = oz.oz_dgemm(handle, ta, tb, m, n, k, 1.0, d, lda, d, ldb, 0.0, d, ldc, oz.prec(7), check=False)
        assert st == pos, (ta, tb, m, n, k, lda, ldb, ldc)
    st = oz.oz_dgemm(handle, "N", "N", 4, 4, 4, 1.0, d, 4, d, 4, 0.0, d, 4, oz.prec(19), check=False)
    assert st == 14
    st = oz.oz_dgemm(handle, "N", "N", 4, 4, 4, 1.0, d, 4, d, 4, 0.0, d, 4, oz.prec(7, kchunk=100), check=False)
    assert st == 14


@pytest.mark.parametrize("cplx", [0, 1])
def test_nonfinite_rows_and_columns_become_nan(oz, handle, cplx):
    rng = np.random.default_rng(4)
    m, n, k = 70, 40, 50
    A, B = wide(rng, (m, k), 5, bool(cplx)), wide(rng, (k, n), 5, bool(cplx))
    A[3, 7] = np.inf
    B[9, 5] = np.nan
    dA, lda = to_dev(A)
    dB, ldb = to_dev(B)
    dC, ldc = to_dev(np.zeros((m, n), A.dtype, order="F"))
    fn = oz.oz_zgemm if cplx else oz.oz_dgemm
    st, rep = fn(handle, "N", "N", m, n, k, 1.0, dA, lda, dB, ldb, 0.0, dC, ldc, oz.prec(6), report=True)
    assert st == 0 and rep.status == oz.OZ_ERR_NONFINITE
    got = from_dev(dC, m, n, ldc)
    bad = np.zeros((m, n), bool)
    bad[3, :] = True
    bad[:, 5] = True
    assert np.all(np.isnan(got[bad]))
    A2, B2 = A.copy(), B.copy()
    A2[3, :] = 0
    B2[:, 5] = 0
    ref = oracle.emu_gemm("N", "N", A2, B2, 6)
    assert np.array_equal(got[~bad], ref[~bad])


def test_subnormal_and_huge_operands(oz, handle):
    rng = np.random.default_rng(5)
    m, n, k = 66, 67, 40
    A = wide(rng, (m, k), 3)
    B = wide(rng, (k, n), 3)
    A[:10] *= 2.0 ** -1050     # subnormal rows
    A[10:20] *= 2.0 ** 900     # huge rows: products overflow to inf with huge B columns
    B[:, :5] *= 2.0 ** 200
    B[:, 5:10] *= 2.0 ** -200  # results underflow into subnormals
    got = run_gemm(oz, handle, 0, "N", "N", A, B, 8)
    want = oracle.emu_gemm("N", "N", A, B, 8)
    assert np.array_equal(got, want, equal_nan=True)


def test_deterministic(oz, handle):
    rng = np.random.default_rng(6)
    A, B = wide(rng, (200, 300), 10, True), wide(rng, (300, 150), 10, True)
    g1 = run_gemm(oz, handle, 1, "N", "N", A, B, 7)
    g2 = run_gemm(oz, handle, 1, "N", "N", A, B, 7)
    assert np.array_equal(np.ascontiguousarray(g1).view(np.float64), np.ascontiguousarray(g2).view(np.float64))


# ----------------------------------------------------------------- full sizes, sampled


def sampled_rows(m, seed, count=6):
    rng = np.random.default_rng(seed)
    return np.unique(np.concatenate([[0, m - 1], rng.integers(0, m, size=count)]))


@pytest.mark.parametrize("n", [2048, 4096])
def test_zgemm_full_size_sampled(oz, handle, n):
    """The benchmark workload (complex, per-row exponents over +-20 binades,
    s = 7) at full size, in the benchmark's launch path; sampled rows of C
    against the oracle, bit for bit."""
    A, B = workloads.zgemm_rowexp(n, seed=0)
    print("zgemm full", n, flush=True)
    got = run_gemm(oz, handle, 1, "N", "N", A, B, 7, zmode=4)
    rows = sampled_rows(n, n)
    want = oracle.emu_gemm("N", "N", A, B, 7, rows=rows)
    assert np.array_equal(got[rows], want)
    ref = oracle.gemm_dd("N", "N", A, B, rows=rows)
    w = np.abs(np.concatenate([A.real, A.imag], axis=1)).max(1)[rows]
    wb = np.abs(np.concatenate([B.real, B.imag], axis=0)).max(0)
    err = oracle.weighted_error(got[rows], ref, w, wb)
    print("zgemm n=%d s=7 sampled rel err %.3g" % (n, err))
    assert err <= 1e-12


def test_dgemm_wide_range_full_size_sampled(oz, handle):
    A, B = workloads.dgemm_wide(4096, 4096, 8192, seed=0)
    print("dgemm wide full", flush=True)
    got = run_gemm(oz, handle, 0, "N", "N", A, B, 8)
    rows = sampled_rows(4096, 1, 4)
    assert np.array_equal(got[rows], oracle.emu_gemm("N", "N", A, B, 8, rows=rows))


# ----------------------------------------------------------------- s above the register-resident range


@pytest.mark.parametrize("cplx", [0, 1])
@pytest.mark.parametrize("s,kc", [(9, 0), (11, 0), (12, 128), (13, 0), (13, 128), (14, 0), (14, 256), (18, 0)])
def test_large_slice_counts_bit_exact(oz, handle, cplx, s, kc):
    rng = np.random.default_rng(100 + s)
    m, n, k = 70, 65, 300
    A, B = wide(rng, (m, k), 40, bool(cplx)), wide(rng, (k, n), 40, bool(cplx))
    print("large s", cplx, s, kc, flush=True)
    got = run_gemm(oz, handle, cplx, "N", "T" if cplx else "N", A, B.T.copy() if cplx else B, s, kc=kc)
    want = oracle.emu_gemm("N", "T" if cplx else "N", A, B.T.copy() if cplx else B, s, kc=kc if kc else None)
    assert np.array_equal(got, want)


def test_large_slice_diagonal_sums_bit_exact(oz, handle):
    rng = np.random.default_rng(9)
    m, n, k, s, kc = 66, 64, 200, 11, 128
    A, B = wide(rng, (m, k), 20), wide(rng, (k, n), 20)
    ra, kpad, nba = oz.oz_split_layout("A", 0, m, k, s)
    rb, _, nbb = oz.oz_split_layout("B", 0, n, k, s)
    dA, lda = to_dev(A)
    dB, ldb = to_dev(B)
    sa = torch.zeros(nba, dtype=torch.int8, device="cuda")
    sb = torch.zeros(nbb, dtype=torch.int8, device="cuda")
    ea = torch.zeros(m, dtype=torch.int32, device="cuda")
    fb = torch.zeros(n, dtype=torch.int32, device="cuda")
    oz.oz_split(handle, "A", "N", 0, m, k, dA, lda, s, ea, sa)
    oz.oz_split(handle, "B", "N", 0, n, k, dB, ldb, s, fb, sb)
    nch = -(-kpad // kc)
    out = torch.zeros(nch * s * rb * ra, dtype=torch.int32, device="cuda")
    oz.oz_diag_sums(handle, s, kc, ra, rb, kpad, sa, sb, out, kernel=0)
    torch.cuda.synchronize()
    got = out.cpu().numpy().reshape(nch, s, rb, ra).transpose(0, 1, 3, 2)
    ref = oracle.diag_sums(oracle.split("A", "N", A, s)[1], oracle.split("B", "N", B, s)[1], s, kc=kc)
    assert np.array_equal(got[:, :, :m, :n], ref)


# ----------------------------------------------------------------- tolerance-driven slice count (a6)

TOL_CASES = [
    ("uniform", 0, 1e-6), ("uniform", 0, 1e-12), ("rowexp", 1, 1e-10), ("rowexp", 1, 1e-14),
    ("wide", 0, 1e-6), ("wide", 0, 1e-10), ("wide", 0, 1e-14), ("spread30", 0, 1e-12),
]


def tol_inputs(kind, cplx, seed=0):
    if kind == "uniform":
        return workloads.dgemm_uniform(150, 130, 170, seed=seed)
    if kind == "rowexp":
        return workloads.zgemm_rowexp(96, seed=seed, m=130, k=110)
    if kind == "wide":
        return workloads.dgemm_wide(140, 120, 260, seed=seed)
    return workloads.dgemm_spread(150, 130, 170, 30, seed=seed)


def scale_weights(A, B):
    if np.iscomplexobj(A):
        return (np.maximum(np.abs(A.real), np.abs(A.imag)).max(1), np.maximum(np.abs(B.real), np.abs(B.imag)).max(0))
    return np.abs(A).max(1), np.abs(B).max(0)


def run_tol(oz, handle, A, B, tol, smax=12, sstart=0, alpha=1.0, beta=0.0, C0=None, kernel=0):
    cplx = np.iscomplexobj(A)
    m, k = A.shape
    n = B.shape[1]
    dA, lda = to_dev(A)
    dB, ldb = to_dev(B)
    C0 = np.zeros((m, n), A.dtype, order="F") if C0 is None else C0
    dC, ldc = to_dev(C0)
    fn = oz.oz_zgemm if cplx else oz.oz_dgemm
    st, rep = fn(handle, "N", "N", m, n, k, alpha, dA, lda, dB, ldb, beta, dC, ldc,
                 oz.prec(0, tol=tol, smax=smax, sstart=sstart, kernel=kernel), report=True)
    assert st == 0 and rep.status == 0
    return from_dev(dC, m, n, ldc), rep


@pytest.mark.parametrize("kind,cplx,tol", TOL_CASES)
def test_tolerance_mode_meets_tol_and_matches_oracle(oz, handle, kind, cplx, tol):
    A, B = tol_inputs(kind, cplx)
    got, rep = run_tol(oz, handle, A, B, tol)
    s1, s0 = rep.slices_used, rep.slices_used - rep.fallbacks
    print("tol %s %g: start %d, used %d, resid %.3g" % (kind, tol, s0, s1, rep.resid_est))
    want = oracle.emu_gemm("N", "N", A, B, s0, s_to=s1, kc=oracle.kchunk(12, bool(cplx)))
    assert np.array_equal(got, want)
    ref = oracle.gemm_dd("N", "N", A, B)
    wa, wb = scale_weights(A, B)
    err = oracle.weighted_error(got, ref, wa, wb)
    # the check stops at half the tolerance, so the true error is within it
    assert err <= tol, (err, tol)
    # the a-posteriori estimate tracks the true weighted error
    assert err / 3 <= rep.resid_est <= 3 * err + 1e-17
    if s1 < 12:
        assert rep.resid_est <= tol / 2


@pytest.mark.parametrize("cplx", [0, 1])
def test_growth_from_a_low_start_is_incremental(oz, handle, cplx):
    A, B = tol_inputs("rowexp" if cplx else "uniform", cplx, seed=3)
    got, rep = run_tol(oz, handle, A, B, 1e-12, sstart=2, alpha=0.5 - 0.25j if cplx else 0.5, beta=0.0)
    assert rep.fallbacks >= 3 and rep.slices_used == 2 + rep.fallbacks
    want = oracle.emu_gemm("N", "N", A, B, 2, s_to=rep.slices_used, kc=oracle.kchunk(12, bool(cplx)),
                           alpha=0.5 - 0.25j if cplx else 0.5)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("kernel", [4, 5])
@pytest.mark.parametrize("cplx,beta", [(0, 0.0), (0, -0.75), (1, 0.0), (1, 0.5 + 0.25j)])
def test_growth_on_two_tile_waves(oz, handle, kernel, cplx, beta):
    # raw writes, top-diagonal growth steps and the final scaling on the blocks
    # whose waves own two 32-row tiles (s <= 6), the 64 x 64 block above
    A, B = tol_inputs("rowexp" if cplx else "uniform", cplx, seed=5)
    rng = np.random.default_rng(9)
    C0 = wide(rng, (A.shape[0], B.shape[1]), 4, bool(cplx))
    print("growth two-tile", kernel, cplx, beta, flush=True)
    got, rep = run_tol(oz, handle, A, B, 1e-13, sstart=2, alpha=1.5, beta=beta, C0=C0, kernel=kernel)
    assert rep.fallbacks >= 3
    want = oracle.emu_gemm("N", "N", A, B, 2, s_to=rep.slices_used, kc=oracle.kchunk(12, bool(cplx)), alpha=1.5,
                           beta=beta, C=C0)
    assert np.array_equal(got, want)


TOL3_CASES = [("rowexp", 1e-10), ("rowexp", 1e-14), ("uniform", 1e-6), ("spread30", 1e-12)]


def tol3_inputs(kind, seed=0):
    """Complex operands: the row-exponent case, or real and imaginary parts
    drawn as two independent real cases."""
    if kind == "rowexp":
        return tol_inputs("rowexp", 1, seed)
    Ar, Br = tol_inputs(kind, 0, seed)
    Ai, Bi = tol_inputs(kind, 0, seed + 100)
    return np.asfortranarray(Ar + 1j * Ai), np.asfortranarray(Br + 1j * Bi)


@pytest.mark.parametrize("kind,tol", TOL3_CASES)
def test_tolerance_mode_3m_meets_tol_and_matches_oracle(oz, handle, kind, tol):
    # the 3-real-product form driven by a tolerance: start from the rule, the
    # check on the combined result, growth of all three products; bit-exact
    # against the oracle's incremental 3M order, the true error within tol
    A, B = tol3_inputs(kind)
    m, k = A.shape
    n = B.shape[1]
    dA, lda = to_dev(A)
    dB, ldb = to_dev(B)
    dC, ldc = to_dev(np.zeros((m, n), np.complex128, order="F"))
    print("tol3 %s %g" % (kind, tol), flush=True)
    st, rep = oz.oz_zgemm(handle, "N", "N", m, n, k, 1.0, dA, lda, dB, ldb, 0.0, dC, ldc,
                          oz.prec(0, tol=tol, zmode=3), report=True)
    assert st == 0 and rep.status == 0 and rep.zmode_used == 3
    s1, s0 = rep.slices_used, rep.slices_used - rep.fallbacks
    print("tol3 %s %g: start %d, used %d, resid %.3g" % (kind, tol, s0, s1, rep.resid_est))
    got = from_dev(dC, m, n, ldc)
    want = oracle.emu_zgemm3("N", "N", A, B, s0, s_to=s1, kc=oracle.kchunk(12))
    assert np.array_equal(got, want)
    ref = oracle.gemm_dd("N", "N", A, B)
    wa, wb = scale_weights(A, B)
    err = oracle.weighted_error(got, ref, wa, wb)
    assert err <= tol, (err, tol)
    assert err / 3 <= rep.resid_est <= 3 * err + 1e-17
    if s1 < 12:
        assert rep.resid_est <= tol / 2


@pytest.mark.parametrize("beta", [0.0, 0.5 - 0.75j])
def test_tolerance_mode_3m_growth_from_low_start(oz, handle, beta):
    A, B = tol_inputs("rowexp", 1, seed=4)
    m, k = A.shape
    n = B.shape[1]
    rng = np.random.default_rng(12)
    C0 = wide(rng, (m, n), 4, True)
    dA, lda = to_dev(A)
    dB, ldb = to_dev(B)
    dC, ldc = to_dev(C0)
    print("tol3 growth beta=%s" % beta, flush=True)
    st, rep = oz.oz_zgemm(handle, "N", "N", m, n, k, 0.75 + 0.5j, dA, lda, dB, ldb, beta, dC, ldc,
                          oz.prec(0, tol=1e-13, sstart=2, zmode=3), report=True)
    assert st == 0 and rep.fallbacks >= 3 and rep.slices_used == 2 + rep.fallbacks
    want = oracle.emu_zgemm3("N", "N", A, B, 2, s_to=rep.slices_used, kc=oracle.kchunk(12), alpha=0.75 + 0.5j,
                             beta=beta, C=C0)
    assert np.array_equal(from_dev(dC, m, n, ldc), want)


def test_tolerance_mode_3m_arguments(oz, handle):
    d = torch.zeros(16, dtype=torch.complex128, device="cuda")
    # balanced digits do not grow incrementally: not in the 3-product form
    st = oz.oz_zgemm(handle, "N", "N", 4, 4, 4, 1.0, d, 4, d, 4, 0.0, d, 4,
                     oz.prec(0, tol=1e-10, zmode=3, digits=1), check=False)
    assert st == 14
    # the workspace query matches the call's plan
    p = oz.prec(0, tol=1e-10, zmode=3)
    assert oz.oz_workspace_size(handle, "N", "N", 300, 200, 100, 1, p) > \
        oz.oz_workspace_size(handle, "N", "N", 300, 200, 100, 1, oz.prec(6, zmode=3))


def test_growth_past_eight_slices_uses_streaming_kernel(oz, handle):
    # tolerance below what 8 slices reach on wide data: the growth goes on with the streaming kernel
    A, B = tol_inputs("wide", 0, seed=4)
    got, rep = run_tol(oz, handle, A, B, 1e-300, smax=11, sstart=7)
    assert rep.slices_used == 11 and rep.fallbacks == 4
    want = oracle.emu_gemm("N", "N", A, B, 7, s_to=11, kc=oracle.kchunk(11))
    assert np.array_equal(got, want)


def test_tolerance_mode_beta_and_nonfinite(oz, handle):
    rng = np.random.default_rng(8)
    A, B = tol_inputs("uniform", 0, seed=5)
    C0 = rng.standard_normal((A.shape[0], B.shape[1]))
    got, rep = run_tol(oz, handle, A, B, 1e-10, alpha=-1.5, beta=0.75, C0=np.asfortranarray(C0))
    s0 = rep.slices_used - rep.fallbacks
    want = oracle.emu_gemm("N", "N", A, B, s0, s_to=rep.slices_used, kc=oracle.kchunk(12), alpha=-1.5, beta=0.75,
                           C=C0)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("kind,cplx", [("uniform", 0), ("rowexp", 1), ("wide", 0), ("spread30", 0)])
def test_select_slices_statistic(oz, handle, kind, cplx):
    A, B = tol_inputs(kind, cplx)
    m, k = A.shape
    n = B.shape[1]
    dA, lda = to_dev(A)
    dB, ldb = to_dev(B)

    def msq(X, axis):
        mx = np.maximum(np.abs(X.real), np.abs(X.imag)).max(axis=axis, keepdims=True)
        E = np.frexp(mx)[1]
        xs = X * np.exp2(-E.astype(float))
        sq = (xs.real ** 2 + xs.imag ** 2) / (2.0 if cplx else 1.0)
        return sq.mean(axis=axis).mean()
    spread = np.sqrt((1 / msq(A, 1) + 1 / msq(B, 0)) / 3)
    for tol in (1e-6, 1e-10, 1e-13):
        s = oz.oz_select_slices(handle, "N", "N", m, n, k, cplx, dA, lda, dB, ldb, tol)
        want = next((t for t in range(1, 13) if 2.5 * (t + 1) * 2.0 ** (-7 * t) * spread <= tol), 12)
        assert s == want, (kind, tol, s, want)


# ----------------------------------------------------------------- 3-real-product complex form


def run_z3(oz, handle, ta, tb, A, B, s, alpha=1.0, beta=0.0, C0=None, kernel=0, kchunk=0, lda_pad=0):
    m = A.shape[0] if ta == "N" else A.shape[1]
    k = A.shape[1] if ta == "N" else A.shape[0]
    n = B.shape[1] if tb == "N" else B.shape[0]
    dA, lda = to_dev(A, A.shape[0] + lda_pad)
    dB, ldb = to_dev(B)
    C0 = np.zeros((m, n), np.complex128, order="F") if C0 is None else C0
    dC, ldc = to_dev(C0, m + 1)
    st, rep = oz.oz_zgemm(handle, ta, tb, m, n, k, alpha, dA, lda, dB, ldb, beta, dC, ldc,
                          oz.prec(s, zmode=3, kernel=kernel, kchunk=kchunk), report=True)
    assert st == 0 and rep.zmode_used == 3
    return from_dev(dC, m, n, ldc), rep


Z3_CASES = [("N", "N", 70, 65, 33, 7, 0), ("T", "C", 130, 70, 257, 5, 1), ("C", "T", 64, 192, 64, 3, 2),
            ("N", "C", 5, 300, 17, 8, 0), ("T", "N", 200, 3, 90, 10, 3), ("C", "N", 33, 47, 2, 1, 0),
            ("N", "T", 150, 130, 300, 7, 2), ("C", "C", 65, 64, 31, 4, 1), ("N", "N", 260, 190, 140, 6, 4),
            ("T", "C", 129, 257, 65, 5, 5), ("C", "N", 300, 70, 33, 8, 4)]


@pytest.mark.parametrize("ta,tb,m,n,k,s,kernel", Z3_CASES)
def test_zgemm_3m_bit_exact(oz, handle, ta, tb, m, n, k, s, kernel):
    rng = np.random.default_rng(m * 7 + n + k)
    A = wide(rng, (m, k) if ta == "N" else (k, m), 12, True)
    B = wide(rng, (k, n) if tb == "N" else (n, k), 12, True)
    C0 = wide(rng, (m, n), 3, True)
    for al, be in ((1.0, 0.0), (0.75 - 0.5j, -1.25 + 0.5j)):
        print("z3", ta, tb, m, n, k, s, kernel, al, be, flush=True)
        got, rep = run_z3(oz, handle, ta, tb, A, B, s, al, be, C0, kernel=kernel, lda_pad=2)
        want = oracle.emu_zgemm3(ta, tb, A, B, s, alpha=al, beta=be, C=C0)
        assert np.array_equal(got, want)


def test_zgemm_3m_chunks_and_nonfinite(oz, handle):
    rng = np.random.default_rng(77)
    A = wide(rng, (40, 700), 8, True)
    B = wide(rng, (700, 30), 8, True)
    got, rep = run_z3(oz, handle, "N", "N", A, B, 6, kchunk=128)
    assert rep.kchunks == 6
    assert np.array_equal(got, oracle.emu_zgemm3("N", "N", A, B, 6, kc=128))
    A[5, 3] = np.inf + 0j
    B[10, 7] = complex(1.0, np.nan)
    got, rep = run_z3(oz, handle, "N", "N", A, B, 6)
    assert rep.status == oz.OZ_ERR_NONFINITE
    bad = np.zeros(got.shape, bool)
    bad[5, :] = True
    bad[:, 7] = True
    assert np.all(np.isnan(got.real[bad])) and np.all(np.isnan(got.imag[bad]))
    # every other entry as if the row / column held zeros
    A2, B2 = A.copy(), B.copy()
    A2[5, :] = 0
    B2[:, 7] = 0
    want = oracle.emu_zgemm3("N", "N", A2, B2, 6)
    assert np.array_equal(got[~bad], want[~bad])


def test_zgemm_3m_full_size_samples(oz, handle):
    """The benchmark product (n = 4096, s = 7) in the 3-product form: sampled
    entries bit-exact, error within the 1e-12 gate against double-double."""
    A, B = workloads.zgemm_rowexp(4096, seed=0)
    got, rep = run_z3(oz, handle, "N", "N", A, B, 7)
    rng = np.random.default_rng(5)
    rows = np.sort(rng.choice(4096, 24, replace=False))
    cols = np.sort(rng.choice(4096, 24, replace=False))
    want = oracle.emu_zgemm3("N", "N", A, B, 7, rows=rows, cols=cols)
    assert np.array_equal(got[np.ix_(rows, cols)], want)
    dd = oracle.gemm_dd("N", "N", A, B, rows=rows, cols=cols)
    wa = np.maximum(np.abs(A.real), np.abs(A.imag)).max(1)[rows]
    wb = np.maximum(np.abs(B.real), np.abs(B.imag)).max(0)[cols]
    err = oracle.weighted_error(got[np.ix_(rows, cols)], dd, wa, wb)
    print("3M n=4096 s=7 sampled weighted error %.3g" % err)
    assert err < 1e-12
