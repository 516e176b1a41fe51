"""Batched products (one persistent GEMM launch per slice count, hipGraph
replay) against the CPU oracle, problem by problem, bit for bit."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from gpu_util import from_dev, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def oz():
    import paper_2503_22875_amd as mod
    return mod


@pytest.fixture(scope="module")
def stream():
    torch.cuda.set_device(0)
    return torch.cuda.Stream()


@pytest.fixture(scope="module")
def handle(oz, stream):
    h = oz.oz_create(0)
    oz.oz_set_stream(h, stream.cuda_stream)
    yield h
    oz.oz_destroy(h)


def make_problem(rng, cplx, m, n, k, ta, tb):
    def mat(r, c):
        x = rng.standard_normal((r, c)) * np.exp2(rng.integers(-8, 9, size=(r, c)))
        if cplx:
            x = x + 1j * rng.standard_normal((r, c)) * np.exp2(rng.integers(-8, 9, size=(r, c)))
        return np.asfortranarray(x)
    A = mat(m, k) if ta == "N" else mat(k, m)
    B = mat(k, n) if tb == "N" else mat(n, k)
    C0 = mat(m, n)
    return A, B, C0


def batch_call(oz, handle, stream, cplx, probs, slices, use_plan=False, replays=0, digits=0, kchunk=0, kernel=0,
               zmode=0):
    dev = []
    for (ta, tb, A, B, C0, al, be) in probs:
        dA, lda = to_dev(A, A.shape[0] + 1)
        dB, ldb = to_dev(B)
        dC, ldc = to_dev(C0)
        dev.append((dA, lda, dB, ldb, dC, ldc))
    torch.cuda.synchronize()
    args = dict(transa=[p[0] for p in probs], transb=[p[1] for p in probs],
                m=[(p[2].shape[0] if p[0] == "N" else p[2].shape[1]) for p in probs],
                n=[(p[3].shape[1] if p[1] == "N" else p[3].shape[0]) for p in probs],
                k=[(p[2].shape[1] if p[0] == "N" else p[2].shape[0]) for p in probs],
                alpha=[p[5] for p in probs], A=[d[0] for d in dev], lda=[d[1] for d in dev],
                B=[d[2] for d in dev], ldb=[d[3] for d in dev], beta=[p[6] for p in probs],
                C=[d[4] for d in dev], ldc=[d[5] for d in dev])
    if not use_plan:
        fn = oz.oz_zgemm_batched if cplx else oz.oz_dgemm_batched
        fn(handle, p=oz.prec(slices if isinstance(slices, int) else 7, digits=digits, kchunk=kchunk, kernel=kernel,
                             zmode=zmode),
           slices=None if isinstance(slices, int) else slices, **args)
    else:
        plan = oz.oz_gemm_batched_plan(handle, cplx, p=oz.prec(slices if isinstance(slices, int) else 7,
                                                               digits=digits, kernel=kernel, zmode=zmode),
                                       slices=None if isinstance(slices, int) else slices, **args)
        oz.oz_batch_graph_launch(plan)
        return plan, dev, args
    stream.synchronize()
    return [from_dev(d[4], args["m"][i], args["n"][i], d[5]) for i, d in enumerate(dev)]


@pytest.mark.parametrize("cplx", [0, 1])
def test_batched_bit_exact_mixed(oz, handle, stream, cplx):
    rng = np.random.default_rng(10 + cplx)
    probs, slices = [], []
    shapes = [(1, 1, 1), (70, 65, 33), (130, 70, 257), (64, 192, 64), (5, 300, 17), (200, 3, 90), (96, 96, 96),
              (33, 47, 2), (0, 5, 5), (6, 0, 4), (7, 8, 0), (40, 30, 20)]
    for i, (m, n, k) in enumerate(shapes):
        ta = "NTC"[i % 3] if cplx else "NT"[i % 2]
        tb = "NCT"[(i // 3) % 3] if cplx else "TN"[i % 2]
        A, B, C0 = make_problem(rng, cplx, m, n, k, ta, tb)
        al = complex(1.0 + 0.1 * i, -0.2 * i) if cplx else 1.0 - 0.1 * i
        be = (complex(0.5, 0.25) if i % 2 else 0.0) if cplx else (0.5 if i % 2 else 0.0)
        if i == len(shapes) - 1:
            al = 0.0  # alpha = 0: C = beta * C
        probs.append((ta, tb, A, B, C0, al, be))
        slices.append(3 + i % 6)
    got = batch_call(oz, handle, stream, cplx, probs, slices)
    for i, (ta, tb, A, B, C0, al, be) in enumerate(probs):
        want = oracle.emu_gemm(ta, tb, A, B, slices[i], alpha=al, beta=be, C=C0) if A.size and B.size else None
        if want is None or al == 0.0:
            m = got[i].shape[0]
            want = (be * C0) if be != 0.0 else np.zeros_like(C0)
            if got[i].size and m:
                assert np.array_equal(got[i], want), i
            continue
        assert np.array_equal(got[i], want), (i, ta, tb, A.shape, B.shape)


@pytest.mark.parametrize("cplx", [0, 1])
@pytest.mark.parametrize("digits", [0, 1])
def test_batched_split_paths(oz, handle, stream, cplx, digits):
    # vectors of at most 1024 doubles (complex k <= 512, real k <= 1024) take
    # the one-pass split, longer ones the scan + digits passes; both at the
    # boundary and past it, every transpose pair, in one batch
    rng = np.random.default_rng(40 + 2 * cplx + digits)
    kmax = 512 if cplx else 1024
    shapes = [(37, 29, kmax), (45, 61, kmax + 1), (9, 130, kmax - 3), (130, 9, kmax + 200), (64, 64, 1)]
    probs = []
    for i, (m, n, k) in enumerate(shapes):
        ta = "NTC"[i % 3] if cplx else "NT"[i % 2]
        tb = "NCT"[(i // 2) % 3] if cplx else "TN"[(i // 2) % 2]
        A, B, C0 = make_problem(rng, cplx, m, n, k, ta, tb)
        be = (complex(0.5, 0.25) if i % 2 else 0.0) if cplx else (0.5 if i % 2 else 0.0)
        probs.append((ta, tb, A, B, C0, 1.25, be))
    print("split paths cplx=%d digits=%d" % (cplx, digits), flush=True)
    got = batch_call(oz, handle, stream, cplx, probs, 6, digits=digits)
    for i, (ta, tb, A, B, C0, al, be) in enumerate(probs):
        want = oracle.emu_gemm(ta, tb, A, B, 6, alpha=al, beta=be, C=C0, balanced=bool(digits))
        assert np.array_equal(got[i], want), (i, ta, tb, A.shape, B.shape)


@pytest.mark.parametrize("cplx", [0, 1])
@pytest.mark.parametrize("s,digits,use_plan", [(6, 0, False), (5, 1, True), (2, 0, False), (7, 0, False)])
def test_batched_two_tile_block(oz, handle, stream, cplx, s, digits, use_plan):
    # the 128 x 64 block of two-tile waves (s <= 6; s = 7 falls back to the
    # 64 x 64 block): ragged shapes across several tiles, every transpose,
    # beta on half of them
    rng = np.random.default_rng(80 + cplx + s)
    shapes = [(130, 70, 257), (257, 129, 40), (64, 192, 64), (5, 300, 17), (300, 5, 90), (129, 65, 33), (1, 1, 1),
              (200, 131, 100)]
    probs = []
    for i, (m, n, k) in enumerate(shapes):
        ta = "NTC"[i % 3] if cplx else "NT"[i % 2]
        tb = "NCT"[(i // 3) % 3] if cplx else "TN"[i % 2]
        A, B, C0 = make_problem(rng, cplx, m, n, k, ta, tb)
        al = complex(0.75, -0.5) if cplx else -1.25
        be = (complex(0.5, 0.25) if i % 2 else 0.0) if cplx else (0.5 if i % 2 else 0.0)
        probs.append((ta, tb, A, B, C0, al, be))
    print("two-tile batch cplx=%d s=%d digits=%d plan=%d" % (cplx, s, digits, use_plan), flush=True)
    if use_plan:
        plan, dev, args = batch_call(oz, handle, stream, cplx, probs, s, use_plan=True, digits=digits, kernel=4)
        try:
            stream.synchronize()
            got = [from_dev(d[4], args["m"][i], args["n"][i], d[5]) for i, d in enumerate(dev)]
        finally:
            oz.oz_batch_destroy(plan)
    else:
        got = batch_call(oz, handle, stream, cplx, probs, s, digits=digits, kernel=4)
    for i, (ta, tb, A, B, C0, al, be) in enumerate(probs):
        want = oracle.emu_gemm(ta, tb, A, B, s, alpha=al, beta=be, C=C0, balanced=bool(digits))
        assert np.array_equal(got[i], want), (i, ta, tb, A.shape, B.shape)


@pytest.mark.parametrize("digits,use_plan,kchunk", [(0, False, 0), (1, True, 0), (0, False, 64), (1, False, 128)])
def test_batched_3m_bit_exact(oz, handle, stream, digits, use_plan, kchunk):
    # the fused 3-real-product tiles: slice counts 1..8 in one batch (s <= 6
    # and s = 7, 8 in two launches), ragged shapes over several tiles, every
    # transpose pair, complex alpha, beta on half of them, forced INT32 chunks
    rng = np.random.default_rng(90 + digits + kchunk)
    shapes = [(70, 65, 33), (130, 70, 257), (64, 192, 64), (5, 300, 17), (200, 3, 90), (96, 96, 96), (33, 47, 2),
              (129, 64, 65), (1, 1, 1), (150, 131, 200)]
    probs, slices = [], []
    for i, (m, n, k) in enumerate(shapes):
        ta, tb = "NTC"[i % 3], "NCT"[(i // 3) % 3]
        A, B, C0 = make_problem(rng, 1, m, n, k, ta, tb)
        al = complex(1.0 - 0.05 * i, 0.1 * (i % 3))
        be = complex(0.5, -0.25) if i % 2 else 0.0
        probs.append((ta, tb, A, B, C0, al, be))
        slices.append(1 + i % 8)
    print("3m batch digits=%d plan=%d kchunk=%d" % (digits, use_plan, kchunk), flush=True)
    if use_plan:
        plan, dev, args = batch_call(oz, handle, stream, 1, probs, slices, use_plan=True, digits=digits, zmode=3)
        try:
            launches, _, _, sl = oz.oz_batch_info(plan, len(probs))
            assert sl == slices and launches == 2
            stream.synchronize()
            got = [from_dev(d[4], args["m"][i], args["n"][i], d[5]) for i, d in enumerate(dev)]
            reps = oz.oz_batch_report(plan, len(probs))
            assert all(r.zmode_used == 3 for r in reps)
        finally:
            oz.oz_batch_destroy(plan)
    else:
        got = batch_call(oz, handle, stream, 1, probs, slices, digits=digits, kchunk=kchunk, zmode=3)
    for i, (ta, tb, A, B, C0, al, be) in enumerate(probs):
        want = oracle.emu_zgemm3(ta, tb, A, B, slices[i], alpha=al, beta=be, C=C0, kc=kchunk or None,
                                 balanced=bool(digits))
        assert np.array_equal(got[i], want), (i, ta, tb, A.shape, B.shape, slices[i])


def test_batched_3m_nonfinite_rows(oz, handle, stream):
    # an Inf in a row of A and a NaN in a column of B: that row and column of
    # C are NaN in both parts, every other entry as if they held zeros
    rng = np.random.default_rng(7)
    probs, bads = [], []
    for i in range(3):
        A, B, C0 = make_problem(rng, 1, 40, 30, 20, "N", "N")
        A, B = A.copy(order="F"), B.copy(order="F")
        r, c = 3 + i, 9 + 2 * i
        A[r, 5] = np.inf + 0j
        B[4, c] = complex(0.0, np.nan)
        probs.append(("N", "N", A, B, C0, 1.0, 0.0))
        bads.append((r, c))
    got = batch_call(oz, handle, stream, 1, probs, 6, zmode=3)
    for i, (ta, tb, A, B, C0, al, be) in enumerate(probs):
        r, c = bads[i]
        bad = np.zeros(got[i].shape, bool)
        bad[r, :] = True
        bad[:, c] = True
        assert np.all(np.isnan(got[i].real[bad])) and np.all(np.isnan(got[i].imag[bad]))
        A2, B2 = A.copy(), B.copy()
        A2[r, :] = 0
        B2[:, c] = 0
        want = oracle.emu_zgemm3(ta, tb, A2, B2, 6)
        assert np.array_equal(got[i][~bad], want[~bad])


@pytest.mark.parametrize("cplx", [0, 1])
@pytest.mark.parametrize("use_plan,kchunk", [(False, 0), (True, 0), (False, 64)])
def test_batched_bit_exact_wide_and_mixed(oz, handle, stream, cplx, use_plan, kchunk):
    # fixed slice counts 1..14 in one batch: s <= 8 share one mixed-s launch,
    # s in 9..12 and 13..14 one wide launch each (with several INT32 chunks:
    # 9..11 and 12, and s = 13, 14 take the streaming body); ragged shapes,
    # every transpose, beta on half of them; as a one-shot call, as a captured
    # plan, and with 64-term chunks
    rng = np.random.default_rng(60 + cplx)
    shapes = [(70, 65, 33), (130, 70, 257), (64, 192, 64), (5, 300, 17), (200, 3, 90), (96, 96, 96), (33, 47, 2),
              (40, 30, 20), (129, 64, 65), (64, 129, 31), (1, 1, 1), (17, 250, 100), (88, 88, 200), (31, 33, 35)]
    probs, slices = [], []
    for i, (m, n, k) in enumerate(shapes):
        ta = "NTC"[i % 3] if cplx else "NT"[i % 2]
        tb = "NCT"[(i // 3) % 3] if cplx else "TN"[i % 2]
        A, B, C0 = make_problem(rng, cplx, m, n, k, ta, tb)
        al = complex(1.0 - 0.05 * i, 0.1) if cplx else 1.0 + 0.1 * i
        be = (complex(0.5, -0.25) if i % 2 else 0.0) if cplx else (0.5 if i % 2 else 0.0)
        probs.append((ta, tb, A, B, C0, al, be))
        slices.append(1 + i)
    print("wide and mixed batch cplx=%d plan=%d kchunk=%d" % (cplx, use_plan, kchunk), flush=True)
    if use_plan:
        plan, dev, args = batch_call(oz, handle, stream, cplx, probs, slices, use_plan=True)
        try:
            launches, _, _, sl = oz.oz_batch_info(plan, len(probs))
            assert sl == slices
            assert launches == 3  # one mixed launch for s <= 8, wide launches for 9..12 and 13..14
            stream.synchronize()
            got = [from_dev(d[4], args["m"][i], args["n"][i], d[5]) for i, d in enumerate(dev)]
        finally:
            oz.oz_batch_destroy(plan)
    else:
        got = batch_call(oz, handle, stream, cplx, probs, slices, kchunk=kchunk)
    for i, (ta, tb, A, B, C0, al, be) in enumerate(probs):
        want = oracle.emu_gemm(ta, tb, A, B, slices[i], alpha=al, beta=be, C=C0, kc=kchunk or None)
        assert np.array_equal(got[i], want), (i, ta, tb, A.shape, B.shape, slices[i])


@pytest.mark.parametrize("cplx", [0, 1])
def test_batched_balanced_bit_exact_mixed(oz, handle, stream, cplx):
    # balanced digits in every problem: slice counts 1..8 mixed (one GEMM
    # launch per count), ragged shapes, every transpose, beta on half of them
    rng = np.random.default_rng(40 + cplx)
    shapes = [(1, 1, 1), (70, 65, 33), (130, 70, 257), (64, 192, 64), (5, 300, 17), (200, 3, 90), (96, 96, 96),
              (33, 47, 2), (7, 8, 0), (40, 30, 20)]
    probs, slices = [], []
    for i, (m, n, k) in enumerate(shapes):
        ta = "NTC"[i % 3] if cplx else "NT"[i % 2]
        tb = "NCT"[(i // 3) % 3] if cplx else "TN"[i % 2]
        A, B, C0 = make_problem(rng, cplx, m, n, k, ta, tb)
        al = complex(1.0 - 0.1 * i, 0.3) if cplx else 1.0 + 0.2 * i
        be = (complex(-0.5, 0.25) if i % 2 else 0.0) if cplx else (0.75 if i % 2 else 0.0)
        probs.append((ta, tb, A, B, C0, al, be))
        slices.append(1 + i % 8)
    print("balanced batch cplx=%d" % cplx, flush=True)
    got = batch_call(oz, handle, stream, cplx, probs, slices, digits=1)
    for i, (ta, tb, A, B, C0, al, be) in enumerate(probs):
        if A.size == 0 or B.size == 0:
            assert np.array_equal(got[i], be * C0 if be != 0.0 else np.zeros_like(C0)), i
            continue
        want = oracle.emu_gemm(ta, tb, A, B, slices[i], alpha=al, beta=be, C=C0, balanced=True)
        assert np.array_equal(got[i], want), (i, ta, tb, A.shape, B.shape, slices[i])


@pytest.mark.parametrize("cplx", [0, 1])
def test_batched_balanced_forced_chunks(oz, handle, stream, cplx):
    # INT32 chunks of 64 terms: every problem folds several chunks with the
    # balanced weights 2^(2-8d) in the persistent kernel
    rng = np.random.default_rng(42 + cplx)
    shapes = [(70, 33, 150), (64, 64, 64), (9, 130, 257), (100, 20, 65)]
    probs, slices = [], []
    for i, (m, n, k) in enumerate(shapes):
        ta = "NC"[i % 2] if cplx else "NT"[i % 2]
        tb = "TN"[i % 2]
        A, B, C0 = make_problem(rng, cplx, m, n, k, ta, tb)
        be = (complex(0.5, -0.5) if cplx else 0.5) if i % 2 else 0.0
        probs.append((ta, tb, A, B, C0, 1.25, be))
        slices.append((4, 6, 8, 5)[i])
    print("balanced batch, kchunk 64, cplx=%d" % cplx, flush=True)
    got = batch_call(oz, handle, stream, cplx, probs, slices, digits=1, kchunk=64)
    for i, (ta, tb, A, B, C0, al, be) in enumerate(probs):
        want = oracle.emu_gemm(ta, tb, A, B, slices[i], alpha=al, beta=be, C=C0, kc=64, balanced=True)
        assert np.array_equal(got[i], want), (i, ta, tb, A.shape, B.shape, slices[i])


def test_batched_balanced_chunk_bound(oz, handle):
    # s = 8: 16384-term chunks fit INT32 with digits up to 127 (bound 16640)
    # but not with balanced digits up to 128 in magnitude (bound 16320)
    d = torch.zeros(16, dtype=torch.complex128, device="cuda")
    base = dict(transa=["N"], transb=["N"], m=[4], n=[4], k=[4], alpha=[1], A=[d], lda=[4], B=[d], ldb=[4],
                beta=[0], C=[d], ldc=[4])
    assert oz.oz_zgemm_batched(handle, check=False, p=oz.prec(8, kchunk=16384, digits=1), **base) == 14
    assert oz.oz_zgemm_batched(handle, check=False, p=oz.prec(8, kchunk=16320, digits=1), **base) == 0
    assert oz.oz_zgemm_batched(handle, check=False, p=oz.prec(8, kchunk=16384), **base) == 0
    torch.cuda.synchronize()


def test_batched_balanced_graph_replay(oz, handle, stream):
    # a captured balanced plan replays with new operands written in place
    rng = np.random.default_rng(41)
    probs = []
    for nb in (48, 130, 64):
        A, B, C0 = make_problem(rng, 0, nb, nb + 3, nb - 5, "N", "T")
        probs.append(("N", "T", A, B, C0, 1.0, 0.0))
    plan, dev, args = batch_call(oz, handle, stream, 0, probs, 6, use_plan=True, digits=1)
    try:
        for rep in range(3):
            stream.synchronize()
            for i, (_, _, A, B, _, _, _) in enumerate(probs):
                A2 = np.asfortranarray(A * (rep + 2) - rep)
                probs[i] = ("N", "T", A2, B, None, 1.0, 0.0)
                dA, lda = dev[i][0], dev[i][1]
                buf = np.zeros((lda, A2.shape[1]), order="F")
                buf[:A2.shape[0]] = A2
                with torch.cuda.stream(stream):
                    dA.copy_(torch.from_numpy(buf.ravel(order="F")))
            oz.oz_batch_graph_launch(plan)
            stream.synchronize()
            for i, (_, _, A2, B, _, _, _) in enumerate(probs):
                got = from_dev(dev[i][4], A2.shape[0], B.shape[0], dev[i][5])
                assert np.array_equal(got, oracle.emu_gemm("N", "T", A2, B, 6, balanced=True)), (rep, i)
    finally:
        oz.oz_batch_destroy(plan)


def test_batched_graph_replays_track_new_inputs(oz, handle, stream):
    rng = np.random.default_rng(20)
    probs = []
    for i, nb in enumerate([32, 96, 64, 160, 128, 32]):
        A, B, C0 = make_problem(rng, 1, nb, nb, nb, "N", "N")
        probs.append(("N", "N", A, B, C0, 1.0, 0.0))
    plan, dev, args = batch_call(oz, handle, stream, 1, probs, 6, use_plan=True)
    try:
        launches, tiles, nbytes, sl = oz.oz_batch_info(plan, len(probs))
        assert launches == 1 and sl == [6] * len(probs)
        for rep in range(3):
            stream.synchronize()
            # eager work between replays: new operands written in place
            for i, (_, _, A, B, _, _, _) in enumerate(probs):
                A2 = np.asfortranarray(A * (rep + 1) + 1j * rep)
                probs[i] = ("N", "N", A2, B, None, 1.0, 0.0)
                dA, lda = dev[i][0], dev[i][1]
                buf = np.zeros((lda, A2.shape[1]), np.complex128, order="F")
                buf[:A2.shape[0]] = A2
                with torch.cuda.stream(stream):
                    dA.copy_(torch.from_numpy(buf.ravel(order="F")))
            if rep:
                oz.oz_batch_graph_launch(plan)
            else:
                oz.oz_batch_execute(plan)
            stream.synchronize()
            for i, (_, _, A2, B, _, _, _) in enumerate(probs):
                got = from_dev(dev[i][4], A2.shape[0], B.shape[1], dev[i][5])
                assert np.array_equal(got, oracle.emu_gemm("N", "N", A2, B, 6)), (rep, i)
    finally:
        oz.oz_batch_destroy(plan)


def test_config3_batch_512_problems(oz, handle, stream):
    """The batched workload: 512 square complex products, n_b = 32 * randint(1, 16),
    s = 6, one persistent launch replayed from a graph; sampled problems bit-exact,
    every problem within the s = 6 error level of the native product."""
    problems = workloads.zgemm_batch(512, seed=0)
    probs = [("N", "N", A, B, np.zeros((A.shape[0], B.shape[1]), np.complex128, order="F"), 1.0, 0.0)
             for A, B in problems]
    plan, dev, args = batch_call(oz, handle, stream, 1, probs, 6, use_plan=True)
    try:
        launches, tiles, nbytes, sl = oz.oz_batch_info(plan, 512)
        print("config3: launches %d tiles %d device %.1f MB" % (launches, tiles, nbytes / 1e6))
        assert launches == 1
        oz.oz_batch_graph_launch(plan)
        stream.synchronize()
        rng = np.random.default_rng(1)
        sample = sorted(set(rng.integers(0, 512, size=8).tolist()) | {0, 511})
        worst = 0.0
        for i, (A, B) in enumerate(problems):
            got = from_dev(dev[i][4], A.shape[0], B.shape[1], dev[i][5])
            if i in sample:
                assert np.array_equal(got, oracle.emu_gemm("N", "N", A, B, 6)), i
            tA = torch.from_numpy(A).cuda()
            tB = torch.from_numpy(B).cuda()
            nat = (tA @ tB).cpu().numpy()
            worst = max(worst, float(np.linalg.norm(got - nat) / np.linalg.norm(nat)))
        print("config3 worst relative error vs native: %.3g" % worst)
        assert worst < 1e-10
    finally:
        oz.oz_batch_destroy(plan)


def test_batched_argument_errors(oz, handle):
    d = torch.zeros(16, dtype=torch.complex128, device="cuda")
    base = dict(transa=["N", "N"], transb=["N", "N"], m=[4, 4], n=[4, 4], k=[4, 4], alpha=[1, 1], A=[d, d],
                lda=[4, 4], B=[d, d], ldb=[4, 4], beta=[0, 0], C=[d, d], ldc=[4, 4])
    for key, val, pos in [("transa", ["N", "X"], 1), ("m", [4, -1], 3), ("lda", [4, 3], 8), ("ldc", [2, 4], 13)]:
        args = dict(base)
        args[key] = val
        assert oz.oz_zgemm_batched(handle, check=False, p=oz.prec(6), **args) == pos
    # fixed slice counts up to 14 (the wide tile from 9 on); 15 and above only tolerance-driven
    assert oz.oz_zgemm_batched(handle, check=False, p=oz.prec(15), **base) == 14
    assert oz.oz_zgemm_batched(handle, check=False, p=oz.prec(14), **base) == 0
    # the 3-real-product form: fixed slice counts up to 8
    assert oz.oz_zgemm_batched(handle, check=False, p=oz.prec(9, zmode=3), **base) == 14
    assert oz.oz_zgemm_batched(handle, check=False, p=oz.prec(0, tol=1e-10, zmode=3), **base) == 14
    assert oz.oz_zgemm_batched(handle, check=False, p=oz.prec(8, zmode=3), **base) == 0
    # a single tolerance-driven 3M call: truncated digits only
    st = oz.oz_zgemm(handle, "N", "N", 4, 4, 4, 1.0, d, 4, d, 4, 0.0, d, 4, oz.prec(0, tol=1e-10, zmode=3, digits=1),
                     check=False)
    assert st == 14
    # balanced digits: fixed slice counts up to 8 only
    assert oz.oz_zgemm_batched(handle, check=False, p=oz.prec(9, digits=1), **base) == 14
    assert oz.oz_zgemm_batched(handle, check=False, p=oz.prec(0, tol=1e-10, digits=1), **base) == 14
    assert oz.oz_zgemm_batched(handle, check=False, p=oz.prec(6, digits=2), **base) == 14


def _tol_batch(oz, handle, stream, cplx, probs, p):
    dev = []
    for (ta, tb, A, B, C0, al, be) in probs:
        dA, lda = to_dev(A, A.shape[0] + 1)
        dB, ldb = to_dev(B)
        dC, ldc = to_dev(C0)
        dev.append((dA, lda, dB, ldb, dC, ldc))
    torch.cuda.synchronize()
    m = [(q[2].shape[0] if q[0] == "N" else q[2].shape[1]) for q in probs]
    n = [(q[3].shape[1] if q[1] == "N" else q[3].shape[0]) for q in probs]
    k = [(q[2].shape[1] if q[0] == "N" else q[2].shape[0]) for q in probs]
    plan = oz.oz_gemm_batched_plan(handle, cplx, [q[0] for q in probs], [q[1] for q in probs], m, n, k,
                                   [q[5] for q in probs], [d[0] for d in dev], [d[1] for d in dev],
                                   [d[2] for d in dev], [d[3] for d in dev], [q[6] for q in probs],
                                   [d[4] for d in dev], [d[5] for d in dev], p=p)
    try:
        oz.oz_batch_execute(plan)
        stream.synchronize()
        reps = oz.oz_batch_report(plan, len(probs))
        with pytest.raises(oz.OzError):
            oz.oz_batch_graph_launch(plan)
    finally:
        oz.oz_batch_destroy(plan)
    got = [from_dev(d[4], m[i], n[i], d[5]) for i, d in enumerate(dev)]
    return got, reps


def _tol_probs(rng, cplx, shapes, beta_every=2):
    probs = []
    for i, (mm, nn, kk) in enumerate(shapes):
        ta = "NTC"[i % 3] if cplx else "NT"[i % 2]
        tb = "NCT"[(i // 2) % 3] if cplx else "TN"[i % 2]
        A, B, C0 = make_problem(rng, cplx, mm, nn, kk, ta, tb)
        al = complex(1.0, -0.5) if cplx else 1.5
        be = (complex(0.25, 0.5) if cplx else -0.5) if i % beta_every == 1 else 0.0
        probs.append((ta, tb, A, B, C0, al, be))
    return probs


def _check_tol_results(probs, got, reps, smax, tol, kc_s):
    for i, (ta, tb, A, B, C0, al, be) in enumerate(probs):
        r = reps[i]
        s1, s0 = r.slices_used, r.slices_used - r.fallbacks
        assert 1 <= s0 <= s1 <= smax, (i, s0, s1)
        # the check stops at half the tolerance unless it ran out of slices
        assert r.resid_est <= tol / 2 or s1 == smax, (i, r.resid_est)
        want = oracle.emu_gemm(ta, tb, A, B, s0, alpha=al, beta=be, C=C0, s_to=s1,
                               kc=oracle.kchunk(kc_s, np.iscomplexobj(A)))
        assert np.array_equal(got[i], want), (i, ta, tb, A.shape, B.shape, s0, s1)


@pytest.mark.parametrize("cplx", [0, 1])
def test_batched_tolerance_rule_matches_oracle(oz, handle, stream, cplx):
    rng = np.random.default_rng(30 + cplx)
    shapes = [(70, 65, 33), (130, 70, 257), (64, 192, 64), (5, 300, 17), (96, 96, 96), (40, 30, 20), (1, 1, 1)]
    probs = _tol_probs(rng, cplx, shapes)
    tol = 1e-11
    got, reps = _tol_batch(oz, handle, stream, cplx, probs, oz.prec(0, tol=tol, smax=12))
    print("rule starts / finals:", [(r.slices_used - r.fallbacks, r.slices_used) for r in reps])
    _check_tol_results(probs, got, reps, 12, tol, 12)


@pytest.mark.parametrize("cplx", [0, 1])
def test_batched_tolerance_growth_from_two(oz, handle, stream, cplx):
    rng = np.random.default_rng(40 + cplx)
    probs = _tol_probs(rng, cplx, [(48, 40, 56), (33, 90, 70), (128, 64, 40)])
    got, reps = _tol_batch(oz, handle, stream, cplx, probs, oz.prec(0, tol=1e-9, smax=8, sstart=2))
    assert all(r.slices_used - r.fallbacks == 2 and r.fallbacks >= 3 for r in reps)
    _check_tol_results(probs, got, reps, 8, 1e-9, 8)


def test_batched_tolerance_growth_past_eight(oz, handle, stream):
    rng = np.random.default_rng(50)
    probs = _tol_probs(rng, 0, [(40, 50, 60), (70, 20, 30)])
    got, reps = _tol_batch(oz, handle, stream, 0, probs, oz.prec(0, tol=1e-300, smax=11, sstart=7))
    assert all(r.slices_used == 11 and r.fallbacks == 4 for r in reps)
    _check_tol_results(probs, got, reps, 11, 1e-300, 11)


@pytest.mark.parametrize("kchunk", [0, 64])
def test_batched_tolerance_growth_to_fourteen(oz, handle, stream, kchunk):
    # growth 11 -> 14 one anti-diagonal per round: the wide launches' ranges
    # 9..12 and 13..14 with one INT32 chunk; with 64-term chunks 12 (several
    # chunks) and the streaming body at 13, 14
    rng = np.random.default_rng(52 + kchunk)
    probs = _tol_probs(rng, 0, [(40, 50, 130), (70, 20, 30), (65, 33, 100)])
    print("growth to 14 kchunk=%d" % kchunk, flush=True)
    got, reps = _tol_batch(oz, handle, stream, 0, probs,
                           oz.prec(0, tol=1e-300, smax=14, sstart=11, kchunk=kchunk))
    assert all(r.slices_used == 14 and r.fallbacks == 3 for r in reps)
    for i, (ta, tb, A, B, C0, al, be) in enumerate(probs):
        want = oracle.emu_gemm(ta, tb, A, B, 11, alpha=al, beta=be, C=C0, s_to=14, kc=kchunk or oracle.kchunk(14))
        assert np.array_equal(got[i], want), (i, A.shape, B.shape)


def test_batched_tolerance_learned_start(oz, handle, stream):
    from oracle import mlp as omlp
    P = {name: np.zeros(shape) for name, shape in omlp.SIZES}
    P["b3"][0] = 4.75
    net = oz.oz_mlp_create(handle, 0)
    oz.oz_mlp_set_params(net, omlp.pack(P).astype(np.float32), np.zeros(16), np.ones(16))
    rng = np.random.default_rng(60)
    probs = _tol_probs(rng, 1, [(48, 40, 56), (96, 96, 96), (17, 130, 45)])
    try:
        with pytest.raises(oz.OzError):  # no selector attached yet
            _tol_batch(oz, handle, stream, 1, probs, oz.prec(0, tol=1e-10, selector=1))
        oz.oz_set_selector(handle, net)
        got, reps = _tol_batch(oz, handle, stream, 1, probs, oz.prec(0, tol=1e-10, selector=1))
        assert all(r.slices_used - r.fallbacks == 5 for r in reps)
        _check_tol_results(probs, got, reps, 12, 1e-10, 12)
    finally:
        oz.oz_set_selector(handle, None)
        oz.oz_mlp_destroy(net)
