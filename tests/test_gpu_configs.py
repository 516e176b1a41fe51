"""The full-size workloads of the benchmark table, checked on sampled entries
against the oracle (the CPU computes only the sampled rows and columns):

* ZGEMM n = 2048 and 4096 with per-row exponents in [-20, 20], s = 3 .. 8, in
  both complex forms and with both digit kinds: sampled entries bit-exact,
  and the scale-weighted error against the double-double product falling by
  about 2^7 per slice, below 1e-12 from s = 7 on (truncated digits) or from
  s = 6 on (balanced digits);
* the benchmark's own configuration -- ZGEMM n = 4096, balanced digits,
  s = 6, both complex forms, launched as the benchmark launches it: a dense
  sample of entries bit-exact and within 1e-12 of the double-double product;
* the wide-range DGEMM 4096 x 8192 x 4096 (rows of A and columns of B scaled
  by 10^U(-8, 8)) driven by the tolerances 1e-6, 1e-10 and 1e-14: the
  residual estimate is within half of each tolerance, the sampled error
  within it, and the result is bit-exact against the oracle's incremental emulation
  from the reported start to the reported final s; and the same DGEMM at
  s = 8 with a forced INT32 split of k into chunks of 2048 terms;
* the complex form zmode 0 picks by size (3 products at 2048^3, 4 below),
  sampled bit-exact against the oracle of that form."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from gpu_util import from_dev

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


def _samples(n, count, seed):
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n, count, replace=False)), np.sort(rng.choice(n, count, replace=False))


@pytest.mark.parametrize("digits", [0, 1])
@pytest.mark.parametrize("n", [2048, 4096])
def test_zgemm_slice_sweep(oz, handle, n, digits):
    A, B = workloads.zgemm_rowexp(n, seed=0)
    dA = torch.from_numpy(A.ravel(order="F")).cuda()
    dB = torch.from_numpy(B.ravel(order="F")).cuda()
    dC = torch.zeros(n * n, dtype=torch.complex128, device="cuda")
    rows, cols = _samples(n, 12, n)
    dd = oracle.gemm_dd("N", "N", A, B, rows=rows, cols=cols)
    wa = np.maximum(np.abs(A.real), np.abs(A.imag)).max(1)[rows]
    wb = np.maximum(np.abs(B.real), np.abs(B.imag)).max(0)[cols]
    errs = {}
    bal = digits == 1
    for zmode in (4, 3):
        for s in range(3, 9):
            print("sweep n=%d zmode=%d digits=%d s=%d" % (n, zmode, digits, s), flush=True)
            oz.oz_zgemm(handle, "N", "N", n, n, n, 1.0, dA, n, dB, n, 0.0, dC, n,
                        oz.prec(s, zmode=zmode, digits=digits))
            torch.cuda.synchronize()
            got = from_dev(dC, n, n, n)[np.ix_(rows, cols)]
            want = (oracle.emu_zgemm3("N", "N", A, B, s, rows=rows, cols=cols, balanced=bal) if zmode == 3
                    else oracle.emu_gemm("N", "N", A, B, s, rows=rows, cols=cols, balanced=bal))
            assert np.array_equal(got, want), (zmode, s)
            errs[zmode, s] = oracle.weighted_error(got, dd, wa, wb)
        print("n=%d zmode=%d digits=%d errors:" % (n, zmode, digits), ["%.2g" % errs[zmode, s] for s in range(3, 9)])
        if not bal:
            for s in range(3, 7):
                assert 2 ** 5 < errs[zmode, s] / errs[zmode, s + 1] < 2 ** 8.5, (zmode, s)
            assert errs[zmode, 7] < 1e-12 and errs[zmode, 6] > 1e-12
        else:
            # balanced digits: about 2^8 per slice (8 bits per digit) down to
            # the FP64 floor, reached near s = 7
            for s in range(3, 6):
                assert 2 ** 6 < errs[zmode, s] / errs[zmode, s + 1] < 2 ** 9.5, (zmode, s)
            assert errs[zmode, 6] < 1e-12 and errs[zmode, 5] > 1e-12
            assert errs[zmode, 8] < 1e-15


@pytest.mark.parametrize("zmode", [3, 4])
def test_zgemm_bench_configuration(oz, handle, zmode):
    # exactly the benchmark's call: n = 4096, per-row exponents +-20, seed 0,
    # s = 6 balanced digits, default kernel, alpha = 1, beta = 0
    n, s = 4096, 6
    A, B = workloads.zgemm_rowexp(n, seed=0)
    dA = torch.from_numpy(A.ravel(order="F")).cuda()
    dB = torch.from_numpy(B.ravel(order="F")).cuda()
    dC = torch.zeros(n * n, dtype=torch.complex128, device="cuda")
    print("bench configuration zmode=%d" % zmode, flush=True)
    oz.oz_zgemm(handle, "N", "N", n, n, n, 1.0, dA, n, dB, n, 0.0, dC, n, oz.prec(s, zmode=zmode, digits=1))
    torch.cuda.synchronize()
    C = from_dev(dC, n, n, n)
    # 48 rows spread over the row blocks (first and last rows included) x 48 columns
    rows, cols = _samples(n, 46, 101)
    rows = np.unique(np.concatenate([[0, n - 1], rows]))
    cols = np.unique(np.concatenate([[0, n - 1], cols]))
    got = C[np.ix_(rows, cols)]
    want = (oracle.emu_zgemm3("N", "N", A, B, s, rows=rows, cols=cols, balanced=True) if zmode == 3
            else oracle.emu_gemm("N", "N", A, B, s, rows=rows, cols=cols, balanced=True))
    assert np.array_equal(got, want)
    dd = oracle.gemm_dd("N", "N", A, B, rows=rows, cols=cols)
    wa = np.maximum(np.abs(A.real), np.abs(A.imag)).max(1)[rows]
    wb = np.maximum(np.abs(B.real), np.abs(B.imag)).max(0)[cols]
    err = oracle.weighted_error(got, dd, wa, wb)
    print("bench configuration zmode=%d: sampled weighted error %.3g" % (zmode, err))
    assert err <= 1e-12
    assert np.all(np.isfinite(C))


@pytest.mark.parametrize("tol", [1e-6, 1e-10, 1e-14])
def test_wide_range_dgemm_tolerance(oz, handle, tol):
    A, B = workloads.dgemm_wide(seed=0)
    m, k = A.shape
    n = B.shape[1]
    dA = torch.from_numpy(A.ravel(order="F")).cuda()
    dB = torch.from_numpy(B.ravel(order="F")).cuda()
    dC = torch.zeros(m * n, dtype=torch.float64, device="cuda")
    print("wide tol %g" % tol, flush=True)
    st, rep = oz.oz_dgemm(handle, "N", "N", m, n, k, 1.0, dA, m, dB, k, 0.0, dC, m, oz.prec(0, tol=tol),
                          report=True)
    assert st == 0 and rep.status == 0
    s0, s1 = rep.slices_used - rep.fallbacks, rep.slices_used
    print("wide tol %g: start %d, final %d, estimate %.3g" % (tol, s0, s1, rep.resid_est))
    rows, cols = _samples(4096, 16, 7)
    got = from_dev(dC, m, n, m)[np.ix_(rows, cols)]
    want = oracle.emu_gemm("N", "N", A, B, s0, s_to=s1, kc=oracle.kchunk(12), rows=rows, cols=cols)
    assert np.array_equal(got, want)
    dd = oracle.gemm_dd("N", "N", A, B, rows=rows, cols=cols)
    err = oracle.weighted_error(got, dd, np.abs(A).max(1)[rows], np.abs(B).max(0)[cols])
    print("wide tol %g: sampled weighted error %.3g" % (tol, err))
    # the check stops at half the tolerance; the true error is within it
    assert rep.resid_est <= tol / 2
    assert err <= tol, (err, tol)


def test_wide_range_dgemm_forced_split_k(oz, handle):
    # the wide-range DGEMM at s = 8 with the INT32 accumulation cut into four
    # chunks of 2048 terms: sampled entries bit-exact against the oracle's
    # chunked FP64 order, and the same error as the one-chunk result
    A, B = workloads.dgemm_wide(seed=0)
    m, k = A.shape
    n = B.shape[1]
    dA = torch.from_numpy(A.ravel(order="F")).cuda()
    dB = torch.from_numpy(B.ravel(order="F")).cuda()
    dC = torch.zeros(m * n, dtype=torch.float64, device="cuda")
    print("wide split-K", flush=True)
    oz.oz_dgemm(handle, "N", "N", m, n, k, 1.0, dA, m, dB, k, 0.0, dC, m, oz.prec(8, kchunk=2048))
    torch.cuda.synchronize()
    rows, cols = _samples(4096, 16, 11)
    got = from_dev(dC, m, n, m)[np.ix_(rows, cols)]
    want = oracle.emu_gemm("N", "N", A, B, 8, kc=2048, rows=rows, cols=cols)
    assert np.array_equal(got, want)
    dd = oracle.gemm_dd("N", "N", A, B, rows=rows, cols=cols)
    err = oracle.weighted_error(got, dd, np.abs(A).max(1)[rows], np.abs(B).max(0)[cols])
    print("wide split-K weighted error %.3g" % err)
    assert err < 1e-14


@pytest.mark.parametrize("k,form", [(2048, 3), (1024, 4)])
def test_default_form_follows_size(oz, handle, k, form):
    # zmode 0: the 3-real-product form once m, n and k are all >= 2048, the
    # 4-product form below; the workspace query agrees with the call
    n = 2048
    rng = np.random.default_rng(k)
    A = np.asfortranarray(rng.standard_normal((n, k)) + 1j * rng.standard_normal((n, k)))
    B = np.asfortranarray(rng.standard_normal((k, n)) + 1j * rng.standard_normal((k, n)))
    dA = torch.from_numpy(A.ravel(order="F")).cuda()
    dB = torch.from_numpy(B.ravel(order="F")).cuda()
    dC = torch.zeros(n * n, dtype=torch.complex128, device="cuda")
    print("default form k=%d" % k, flush=True)
    p = oz.prec(6, digits=1)
    st, rep = oz.oz_zgemm(handle, "N", "N", n, n, k, 1.0, dA, n, dB, k, 0.0, dC, n, p, report=True)
    assert st == 0 and rep.zmode_used == form
    assert oz.oz_workspace_size(handle, "N", "N", n, n, k, 1, p) == \
        oz.oz_workspace_size(handle, "N", "N", n, n, k, 1, oz.prec(6, digits=1, zmode=form))
    rows, cols = _samples(n, 10, k + 1)
    got = from_dev(dC, n, n, n)[np.ix_(rows, cols)]
    want = (oracle.emu_zgemm3("N", "N", A, B, 6, rows=rows, cols=cols, balanced=True) if form == 3
            else oracle.emu_gemm("N", "N", A, B, 6, rows=rows, cols=cols, balanced=True))
    assert np.array_equal(got, want)
