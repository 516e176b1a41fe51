"""Pins of the selector oracle (features, error table, labels) and of the
shared counter-based instance generator, on the CPU."""
import numpy as np
import pytest

import oracle
import workloads
from oracle import select as osel


def test_splitmix64_published_values():
    # splitmix64 seeded with 1234567: the first outputs as published with the
    # reference implementation (Vigna, prng.di.unimi.it/splitmix64.c)
    want = [6457827717110365317, 3203168211198807973, 9817491932198370423, 4593380528125082431,
            16408922859458223821]
    got = [int(workloads.draw(1234567, c)) for c in range(5)]
    assert got == want


def test_generator_structure():
    p = dict(m=40, n=24, k=56, sig_el=0, sig_vec=0, bits=53, family=0, zero_q=0, key=7)
    A, B = workloads.gen_operands(p)
    assert A.shape == (40, 56) and B.shape == (56, 24)
    assert A.flags.f_contiguous and B.flags.f_contiguous
    # family 0, no spread: |x| in [1/2, 1), both signs
    for X in (A, B):
        assert np.all((np.abs(X) >= 0.5) & (np.abs(X) < 1.0))
        assert 0.3 < np.mean(X > 0) < 0.7
    # bit truncation: every entry a multiple of 2^-(bits) at exponent 0
    q = dict(p, bits=9)
    A9, _ = workloads.gen_operands(q)
    assert np.all(np.ldexp(A9, 9) == np.round(np.ldexp(A9, 9)))
    # same significand prefix as the untruncated draw
    assert np.all(np.abs(A - A9) < 2.0 ** -9)
    # zero fraction close to zero_q / 2^24
    z = dict(p, zero_q=1 << 23)
    Az, Bz = workloads.gen_operands(z)
    assert 0.4 < np.mean(Az == 0) < 0.6
    assert np.array_equal(Az != 0, Az != 0) and np.all((Az == 0) | (Az == A))
    # vector exponent spread: constant per row of A, per column of B
    v = dict(p, sig_vec=10)
    Av, Bv = workloads.gen_operands(v)
    ra = np.log2(np.abs(Av) / np.abs(A))
    rb = np.log2(np.abs(Bv) / np.abs(B))
    assert np.all(ra == ra[:, :1]) and np.all(rb == rb[:1, :])
    assert ra.min() >= -5 and ra.max() <= 5 and len(np.unique(ra)) > 3
    # element spread: integer exponent offsets in [-sig//2, sig - sig//2]
    e = dict(p, sig_el=7)
    Ae, _ = workloads.gen_operands(e)
    re = np.log2(np.abs(Ae) / np.abs(A))
    assert np.all(re == np.round(re)) and re.min() == -3 and re.max() == 4
    # bell family: values in (-2, 2), more mass near 0 than at the edges
    Ab, _ = workloads.gen_operands(dict(p, family=1))
    assert np.all(np.abs(Ab) < 2.0) and np.mean(np.abs(Ab) < 0.5) > np.mean(np.abs(Ab) > 1.0)


def test_instance_table():
    ps, tols = workloads.selector_instances(200, seed=3)
    dims = np.array([[p["m"], p["n"], p["k"]] for p in ps])
    assert dims.min() >= 64 and dims.max() <= 2048 and np.all(dims % 16 == 0)
    assert tols.shape == (200, 4) and tols.min() >= 1e-15 and tols.max() <= 1e-4
    sig = np.array([p["sig_el"] + p["sig_vec"] for p in ps])
    assert sig.min() >= 0 and sig.max() <= 40


def _hand_features():
    # row 0: 1, 1/2, 1/4, 0  -> E = 1; gaps 0,1,2; widths 1,2,3
    # row 1: 3, -3/2, 3/4, 3/8 -> E = 2; gaps 0,1,2,3; widths 2,3,4,5
    A = np.asfortranarray([[1.0, 0.5, 0.25, 0.0], [3.0, -1.5, 0.75, 0.375]])
    return A


def test_side_stats_closed_form():
    A = _hand_features()
    z, gm, gs, g90, wm, w90, M = osel.side_stats("A", "N", A)
    g = np.array([0, 1, 2, 0, 1, 2, 3.0])
    assert z == 1.0 / 8.0
    assert gm == pytest.approx(9.0 / 7.0, rel=1e-15)
    assert gs == pytest.approx(np.sqrt(np.mean((g - 9.0 / 7.0) ** 2)), rel=1e-14)
    assert g90 == 3.0
    assert wm == pytest.approx(20.0 / 7.0, rel=1e-15)
    assert w90 == 5.0
    # mean squares of x 2^-E: row 0 (1/2, 1/4, 1/8, 0), row 1 (3/4, 3/8, 3/16, 3/32)
    r0 = (0.25 + 1 / 16 + 1 / 64) / 4
    r1 = (9 / 16 + 9 / 64 + 9 / 256 + 9 / 1024) / 4
    assert M == pytest.approx((r0 + r1) / 2, rel=1e-15)
    # the same matrix seen as op(B) columns ('T' of the transpose is the rows again)
    assert osel.side_stats("B", "T", A) == osel.side_stats("A", "N", A)
    assert osel.side_stats("B", "N", np.asfortranarray(A.T)) == osel.side_stats("A", "N", A)


def test_side_stats_complex_parts_and_caps():
    # 1 + 2i: parts 1 (gap 1, width 2) and 2 (gap 0, width 1) under E = 2
    z, gm, gs, g90, wm, w90, M = osel.side_stats("A", "N", np.array([[1.0 + 2.0j]]))
    assert (z, gm, g90, wm, w90) == (0.0, 0.5, 1.0, 1.5, 2.0)
    assert M == pytest.approx((0.0625 + 0.25) / 2, rel=1e-15)
    # a gap of 200 binades and a subnormal entry are capped at 127
    A = np.array([[1.0, 2.0 ** -200, 3 * 2.0 ** -1074]])
    z, gm, gs, g90, wm, w90, M = osel.side_stats("A", "N", A)
    assert gm == pytest.approx((0 + 127 + 127) / 3)
    assert g90 == 127 and w90 == 127
    # 3 * 2^-1074: significand 3 (two bits)
    A = np.array([[2.0 ** -1070, 3 * 2.0 ** -1074]])
    _, gm, _, _, wm, _, _ = osel.side_stats("A", "N", A)
    assert gm == pytest.approx((0 + 3) / 2) and wm == pytest.approx((1 + 5) / 2)


def test_features_invariances():
    rng = np.random.default_rng(5)
    A = np.asfortranarray(rng.standard_normal((30, 20)) * np.exp2(rng.integers(-6, 7, (30, 20))))
    B = np.asfortranarray(rng.standard_normal((20, 25)) * np.exp2(rng.integers(-6, 7, (20, 25))))
    f = osel.features("N", "N", A, B, 1e-10)
    assert f.shape == (16,)
    # row scaling by powers of two and permutations inside a vector leave it unchanged
    D = np.exp2(rng.integers(-30, 30, 30))
    A2 = np.asfortranarray(A * D[:, None])
    A2 = np.asfortranarray(A2[:, rng.permutation(20)])
    assert np.allclose(osel.features("N", "N", A2, B, 1e-10), f, rtol=1e-13, atol=0)
    # transposed storage gives the same features
    assert np.allclose(osel.features("T", "T", np.asfortranarray(A.T), np.asfortranarray(B.T), 1e-10), f,
                       rtol=0, atol=0)
    # globals
    assert f[12] == pytest.approx(np.log2(20)) and f[13] == pytest.approx(0.5 * np.log2(30 * 25))
    assert f[14] == pytest.approx(10.0)
    # complex: stacked real product has 2k terms
    fz = osel.features("N", "N", A + 1j * A, B + 1j * B, 1e-10)
    assert fz[12] == pytest.approx(np.log2(40))


def test_eps_table_exact_integers():
    # integer entries with every row / column max in [64, 127]: s = 1 is exact
    rng = np.random.default_rng(2)
    A = rng.integers(-127, 128, (24, 40)).astype(np.float64)
    B = rng.integers(-127, 128, (40, 16)).astype(np.float64)
    A[:, 0] = 100.0
    B[0, :] = -90.0
    A, B = np.asfortranarray(A), np.asfortranarray(B)
    eps = osel.eps_table("N", "N", A, B, s_ref=6)
    assert all(eps[s] == 0.0 for s in range(1, 7))
    assert osel.label(eps, 1e-15, smax=6) == 2


def test_eps_table_decay_and_labels():
    A, B = workloads.dgemm_uniform(48, 40, 56, seed=4)
    eps = osel.eps_table("N", "N", A, B, s_ref=9)
    # geometric decay of about 2^6.6 per slice (Table 1) while above the FP64 floor
    for s in range(2, 7):
        assert 2 ** 5 < eps[s] / eps[s + 1] < 2 ** 8.5, s
    # error against the exact (double-double) product agrees with the table
    Cdd = oracle.gemm_dd("N", "N", A, B)
    wa, wb = osel.weights("N", "N", A, B)
    for s in (3, 5):
        e_true = osel.weighted_eps(oracle.emu_gemm("N", "N", A, B, s), Cdd, wa, wb)
        assert e_true == pytest.approx(eps[s], rel=1e-6)
    # label: smallest passing s, non-increasing in the tolerance
    tols = np.logspace(-16, -2, 40)
    labs = [osel.label(eps, t, smax=9) for t in tols]
    assert all(a >= b for a, b in zip(labs, labs[1:]))
    for t, lab in zip(tols, labs):
        assert eps[lab] <= t or lab == 9
        assert lab == 2 or eps[lab - 1] > t
