"""Parity of the learned slice-count selection (through the C ABI) with the
CPU oracle: generator bit for bit, features and error tables to floating-point
tolerance, labels exact, the network's forward pass, gradient and Adam step
against the float64 oracle network, and the learned start of a
tolerance-driven call against the oracle's incremental emulation."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from gpu_util import from_dev, to_dev
from oracle import mlp as omlp
from oracle import select as osel

pytestmark = pytest.mark.gpu

# float32 features against the float64 definition
FEAT_RTOL, FEAT_ATOL = 2e-6, 2e-6


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


GEN_CASES = [
    dict(m=70, n=33, k=45, sig_el=0, sig_vec=0, bits=53, family=0, zero_q=0, key=1),
    dict(m=64, n=64, k=64, sig_el=17, sig_vec=0, bits=53, family=1, zero_q=0, key=2),
    dict(m=5, n=130, k=97, sig_el=6, sig_vec=23, bits=9, family=0, zero_q=1 << 22, key=3),
    dict(m=129, n=1, k=3, sig_el=40, sig_vec=40, bits=1, family=1, zero_q=(1 << 24) - 1, key=2 ** 63 + 5),
]


@pytest.mark.parametrize("case", range(len(GEN_CASES)))
def test_generator_bit_exact(oz, handle, case):
    p = GEN_CASES[case]
    A, B = workloads.gen_operands(p)
    lda, ldb = p["m"] + 3, p["k"] + 1
    dA = torch.full((lda * p["k"],), np.nan, dtype=torch.float64, device="cuda")
    dB = torch.full((ldb * p["n"],), np.nan, dtype=torch.float64, device="cuda")
    oz.oz_gen_operands(handle, p, dA, lda, dB, ldb)
    torch.cuda.synchronize()
    gA = from_dev(dA, p["m"], p["k"], lda)
    gB = from_dev(dB, p["k"], p["n"], ldb)
    assert np.array_equal(gA.view(np.uint64), A.view(np.uint64))
    assert np.array_equal(gB.view(np.uint64), B.view(np.uint64))
    # padding rows untouched
    assert np.all(np.isnan(dA.cpu().numpy().reshape(p["k"], lda)[:, p["m"]:]))


def _feature_inputs(kind):
    rng = np.random.default_rng(hash(kind) % 1000)
    if kind == "uniform":
        A, B = workloads.dgemm_uniform(150, 90, 200, seed=1)
        return "N", "N", A, B
    if kind == "spread":
        A, B = workloads.dgemm_spread(96, 130, 70, 30, seed=2)
        return "T", "N", np.asfortranarray(A.T), B
    if kind == "zeros_short":
        p = dict(m=100, n=80, k=140, sig_el=12, sig_vec=5, bits=11, family=1, zero_q=1 << 23, key=9)
        A, B = workloads.gen_operands(p)
        A[3, :] = 0.0                    # an all-zero row
        return "N", "T", A, np.asfortranarray(B.T)
    if kind == "complex":
        A, B = workloads.zgemm_rowexp(n=72, seed=3, m=50, k=90)
        return "C", "N", np.asfortranarray(A.conj().T), B
    if kind == "subnormal":
        A = np.asfortranarray(rng.standard_normal((40, 33)) * 2.0 ** -1060)
        B = np.asfortranarray(rng.standard_normal((33, 20)))
        return "N", "N", A, B
    raise ValueError(kind)


@pytest.mark.parametrize("kind", ["uniform", "spread", "zeros_short", "complex", "subnormal"])
def test_features_match_oracle(oz, handle, kind):
    ta, tb, A, B = _feature_inputs(kind)
    cplx = np.iscomplexobj(A)
    m = A.shape[0] if ta == "N" else A.shape[1]
    k = A.shape[1] if ta == "N" else A.shape[0]
    n = B.shape[1] if tb == "N" else B.shape[0]
    dA, lda = to_dev(A, A.shape[0] + 2)
    dB, ldb = to_dev(B)
    tols = [1e-4, 3.3e-9, 1e-15]
    feat = torch.zeros(len(tols) * 16, dtype=torch.float32, device="cuda")
    s_rule = oz.oz_features(handle, ta, tb, m, n, k, cplx, dA, lda, dB, ldb, tols, feat)
    got = feat.cpu().numpy().reshape(len(tols), 16).astype(np.float64)
    for t, tol in enumerate(tols):
        want = osel.features(ta, tb, A, B, tol)
        np.testing.assert_allclose(got[t], want, rtol=FEAT_RTOL, atol=FEAT_ATOL, err_msg="%s tol %g" % (kind, tol))
        # the rule's choice from the same statistics
        Ma = osel.side_stats("A", ta, A)[6]
        Mb = osel.side_stats("B", tb, B)[6]
        spread = np.sqrt((1 / Ma + 1 / Mb) / 3)
        rule = next((s for s in range(1, 13) if 2.5 * (s + 1) * 2.0 ** (-7 * s) * spread <= tol), 12)
        assert s_rule[t] == rule


def test_dataset_matches_oracle(oz, handle):
    """Error tables, features and labels of GPU-generated instances, against the
    oracle run on the same instances drawn by the CPU generator."""
    params = [
        dict(m=80, n=48, k=96, sig_el=0, sig_vec=0, bits=53, family=1, zero_q=0, key=11),
        dict(m=33, n=70, k=50, sig_el=30, sig_vec=0, bits=53, family=0, zero_q=0, key=12),
        dict(m=64, n=64, k=130, sig_el=4, sig_vec=20, bits=13, family=1, zero_q=1 << 22, key=13),
        dict(m=17, n=29, k=1, sig_el=2, sig_vec=2, bits=53, family=0, zero_q=0, key=14),
    ]
    tols = np.array([[1e-4, 1e-8, 1e-12, 1e-15]] * len(params))
    s_ref = 10
    rows = len(params) * tols.shape[1]
    X = torch.zeros(rows * 16, dtype=torch.float32, device="cuda")
    y = torch.zeros(rows, dtype=torch.float32, device="cuda")
    s_rule, eps = oz.oz_selector_dataset(handle, params, tols, X, y, s_ref=s_ref)
    Xh = X.cpu().numpy().reshape(rows, 16).astype(np.float64)
    yh = y.cpu().numpy()
    for b, p in enumerate(params):
        A, B = workloads.gen_operands(p)
        want = osel.eps_table("N", "N", A, B, s_ref=s_ref)
        for s in range(1, s_ref + 1):
            assert eps[b][s - 1] == pytest.approx(want[s], rel=1e-9, abs=1e-300), (b, s)
        for t in range(tols.shape[1]):
            r = b * tols.shape[1] + t
            np.testing.assert_allclose(Xh[r], osel.features("N", "N", A, B, tols[b, t]), rtol=FEAT_RTOL,
                                       atol=FEAT_ATOL)
            lab = osel.label(want, tols[b, t], smax=s_ref)
            # a label may differ only where eps sits at the tolerance itself
            near = any(abs(want[s] / tols[b, t] - 1) < 1e-9 for s in range(2, s_ref))
            assert yh[r] == lab or near, (b, t, yh[r], lab)


def _net(seed, rows):
    rng = np.random.default_rng(seed)
    p = (rng.standard_normal(omlp.NPARAM) * 0.3).astype(np.float32)
    X = (rng.standard_normal((rows, 16)) * 2.0 + 1.0).astype(np.float32)
    t = rng.integers(2, 13, rows).astype(np.float32)
    mu = (rng.standard_normal(16) * 0.5).astype(np.float32)
    sd = rng.uniform(0.5, 2.0, 16).astype(np.float32)
    return p, X, t, mu, sd


def _upload_net(oz, handle, p, mu, sd):
    net = oz.oz_mlp_create(handle, 0)
    oz.oz_mlp_set_params(net, p, mu, sd)
    return net


def test_mlp_forward_and_gradient(oz, handle):
    rows = 70
    p, X, t, mu, sd = _net(1, rows)
    net = _upload_net(oz, handle, p, mu, sd)
    try:
        dX = torch.from_numpy(X.ravel()).cuda()
        dt = torch.from_numpy(t).cuda()
        y = torch.zeros(rows, dtype=torch.float32, device="cuda")
        oz.oz_mlp_forward(net, rows, dX, y)
        want, _ = omlp.forward(p.astype(np.float64), X.astype(np.float64), mu.astype(np.float64),
                               sd.astype(np.float64))
        got = y.cpu().numpy().astype(np.float64)
        assert np.max(np.abs(got - want)) <= 1e-5 * max(1.0, np.max(np.abs(want)))
        g, loss = oz.oz_mlp_grad(net, rows, dX, dt, 0.9)
        lw, gw = omlp.loss_grad(p.astype(np.float64), X.astype(np.float64), t.astype(np.float64), 0.9,
                                mu.astype(np.float64), sd.astype(np.float64))
        assert loss == pytest.approx(lw, rel=1e-5)
        g = np.asarray(g, np.float64)
        assert np.max(np.abs(g - gw)) <= 1e-5 * np.max(np.abs(gw))
        # one Adam step from a fresh optimiser state
        lr = 1e-3
        oz.oz_mlp_train_step(net, rows, dX, dt, 0.9, lr)
        p1 = np.asarray(oz.oz_mlp_get_params(net)[0], np.float64)
        pw, _, _ = omlp.adam_step(p.astype(np.float64), gw, np.zeros(omlp.NPARAM), np.zeros(omlp.NPARAM), 1, lr)
        # the first step is lr * g / (|g| + eps): compare where the gradient is not tiny
        big = np.abs(gw) > 1e-3 * np.max(np.abs(gw))
        assert np.max(np.abs(p1 - pw)[big]) <= 1e-6 + 1e-6 * np.max(np.abs(pw))
        assert np.max(np.abs(p1 - pw)) <= 2 * lr
    finally:
        oz.oz_mlp_destroy(net)


def test_mlp_training_fits_and_round_trips(oz, handle, tmp_path):
    # a smooth target the network can fit: t = 2 + 0.5 * |x0 - x1| + x2^2 / 4
    rng = np.random.default_rng(7)
    rows = 4096
    X = rng.standard_normal((rows, 16)).astype(np.float32)
    t = (2 + 0.5 * np.abs(X[:, 0] - X[:, 1]) + X[:, 2] ** 2 / 4).astype(np.float32)
    dX = torch.from_numpy(X.ravel()).cuda()
    dt = torch.from_numpy(t).cuda()
    net = oz.oz_mlp_create(handle, 123)
    try:
        oz.oz_mlp_fit_norm(net, rows, dX)
        _, mu, sd = oz.oz_mlp_get_params(net)
        assert np.allclose(mu, X.mean(0), atol=1e-4) and np.allclose(sd, X.std(0), rtol=1e-4)
        losses = oz.oz_mlp_train(net, rows, dX, dt, epochs=30, batch=128, tau=0.5, lr=3e-3, seed=5)
        print("losses", losses[0], losses[-1])
        assert losses[-1] < 0.25 * losses[0]
        # deterministic: the same seed from the same start gives the same network
        net2 = oz.oz_mlp_create(handle, 123)
        oz.oz_mlp_fit_norm(net2, rows, dX)
        losses2 = oz.oz_mlp_train(net2, rows, dX, dt, epochs=30, batch=128, tau=0.5, lr=3e-3, seed=5)
        assert losses2 == losses
        assert oz.oz_mlp_get_params(net2) == oz.oz_mlp_get_params(net)
        oz.oz_mlp_destroy(net2)
        path = str(tmp_path / "net.bin")
        oz.oz_mlp_save(net, path)
        net3 = oz.oz_mlp_load(handle, path)
        y1 = torch.zeros(rows, dtype=torch.float32, device="cuda")
        y3 = torch.zeros(rows, dtype=torch.float32, device="cuda")
        oz.oz_mlp_forward(net, rows, dX, y1)
        oz.oz_mlp_forward(net3, rows, dX, y3)
        assert torch.equal(y1, y3)
        oz.oz_mlp_destroy(net3)
    finally:
        oz.oz_mlp_destroy(net)


def test_learned_start_in_tolerance_mode(oz, handle):
    """A hand-set network that always answers 3.75 (so s = 4): the call starts at
    4, grows incrementally, and gives the oracle's incremental result."""
    P = {name: np.zeros(shape) for name, shape in omlp.SIZES}
    P["b3"][0] = 3.75
    net = _upload_net(oz, handle, omlp.pack(P).astype(np.float32), np.zeros(16, np.float32),
                      np.ones(16, np.float32))
    try:
        with pytest.raises(oz.OzError):
            A0 = torch.zeros(4, dtype=torch.float64, device="cuda")
            oz.oz_predict_slices(handle, "N", "N", 2, 2, 2, 0, A0, 2, A0, 2, 1e-10)
        oz.oz_set_selector(handle, net)
        A, B = workloads.dgemm_uniform(130, 70, 96, seed=8)
        dA, lda = to_dev(A)
        dB, ldb = to_dev(B)
        assert oz.oz_predict_slices(handle, "N", "N", 130, 70, 96, 0, dA, lda, dB, ldb, 1e-12) == 4
        dC, ldc = to_dev(np.zeros((130, 70), order="F"))
        st, rep = oz.oz_dgemm(handle, "N", "N", 130, 70, 96, 1.0, dA, lda, dB, ldb, 0.0, dC, ldc,
                              oz.prec(0, tol=1e-12, selector=1), report=True)
        assert rep.slices_used - rep.fallbacks == 4 and rep.fallbacks >= 2
        want = oracle.emu_gemm("N", "N", A, B, 4, s_to=rep.slices_used, kc=oracle.kchunk(12))
        assert np.array_equal(from_dev(dC, 130, 70, ldc), want)
        # complex product through the same selector
        Az, Bz = workloads.zgemm_rowexp(n=40, seed=9, m=36, k=52)
        dA, lda = to_dev(Az)
        dB, ldb = to_dev(Bz)
        dC, ldc = to_dev(np.zeros((36, 40), np.complex128, order="F"))
        st, rep = oz.oz_zgemm(handle, "N", "N", 36, 40, 52, 1.0, dA, lda, dB, ldb, 0.0, dC, ldc,
                              oz.prec(0, tol=1e-9, selector=1), report=True)
        assert rep.slices_used - rep.fallbacks == 4
        want = oracle.emu_gemm("N", "N", Az, Bz, 4, s_to=rep.slices_used, kc=oracle.kchunk(12, True))
        assert np.array_equal(from_dev(dC, 36, 40, ldc), want)
        # and in the 3-real-product form
        st, rep = oz.oz_zgemm(handle, "N", "N", 36, 40, 52, 1.0, dA, lda, dB, ldb, 0.0, dC, ldc,
                              oz.prec(0, tol=1e-9, selector=1, zmode=3), report=True)
        assert rep.slices_used - rep.fallbacks == 4 and rep.zmode_used == 3
        want = oracle.emu_zgemm3("N", "N", Az, Bz, 4, s_to=rep.slices_used, kc=oracle.kchunk(12))
        assert np.array_equal(from_dev(dC, 36, 40, ldc), want)
    finally:
        oz.oz_set_selector(handle, None)
        oz.oz_mlp_destroy(net)


def test_predicted_slices_match_oracle_network(oz, handle):
    rng = np.random.default_rng(4)
    p = (rng.standard_normal(omlp.NPARAM) * 0.2).astype(np.float32)
    mu = np.array([0.1, 3, 2, 6, 30, 40, 0.1, 3, 2, 6, 30, 40, 8, 8, 9, -1], np.float32)
    sd = np.array([0.2, 2, 2, 4, 10, 10, 0.2, 2, 2, 4, 10, 10, 2, 2, 3, 2], np.float32)
    net = _upload_net(oz, handle, p, mu, sd)
    oz.oz_set_selector(handle, net)
    try:
        checked = 0
        for seed in range(6):
            A, B = workloads.dgemm_spread(60 + 10 * seed, 50, 70, 5 * seed, seed=seed)
            dA, lda = to_dev(A)
            dB, ldb = to_dev(B)
            for tol in (1e-6, 1e-11, 1e-14):
                s = oz.oz_predict_slices(handle, "N", "N", A.shape[0], 50, 70, 0, dA, lda, dB, ldb, tol, smax=12)
                f = osel.features("N", "N", A, B, tol).astype(np.float32).astype(np.float64)
                yv, _ = omlp.forward(p.astype(np.float64), f[None, :], mu.astype(np.float64), sd.astype(np.float64))
                if abs((yv[0] - 0.5) - round(yv[0] - 0.5)) < 1e-3:
                    continue  # too close to a half-integer for float32 to decide the rounding
                assert s == omlp.predict_slices(yv, 2, 12)[0]
                checked += 1
        assert checked >= 12
    finally:
        oz.oz_set_selector(handle, None)
        oz.oz_mlp_destroy(net)




def _selection_gain(oz, kind):
    import bench
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    h = oz.oz_create(0)
    oz.oz_set_stream(h, stream.cuda_stream)
    net = None
    try:
        oz.oz_load_tuning(h)
        net = oz.oz_mlp_load(h)
        oz.oz_set_selector(h, net)
        print("gain: drawing the %s batch" % kind, flush=True)
        dev, ns, tols, _ = bench.mixed_batch_on_device(oz, h, 512, seed=0, kind=kind)
        print("gain: running fixed / rule / escalate / learned", flush=True)
        out = bench.selection_gain(oz, h, stream, dev, ns, tols, steps=5, warmup=1)
        print(out, flush=True)
        for way in ("fixed", "rule", "escalate", "learned"):
            assert out[way]["pass_true"] == 1.0, way
        return out
    finally:
        oz.oz_set_selector(h, None)
        if net is not None:
            oz.oz_mlp_destroy(net)
        oz.oz_destroy(h)


def test_learned_selection_gain_instance_distribution(oz):
    # 512 problems of the batched workload's sizes, each with its own
    # structure drawn from the selector's instance distribution and its own
    # tolerance in [1e-15, 1e-4]: every way of choosing s meets every
    # problem's tolerance by its true error (judged by the s = 12 emulation);
    # the learned start spends less INT8 work than the rule and than the
    # smallest single fixed s that passes every problem, and less time than
    # that fixed s and than escalation from s = 2 (best of 5 executions).
    out = _selection_gain(oz, "mixed")
    assert out["learned"]["int8_tops"] < out["rule"]["int8_tops"] < out["fixed"]["int8_tops"]
    assert out["learned"]["ms_min"] < out["fixed"]["ms_min"]
    assert out["learned"]["ms_min"] < out["escalate"]["ms_min"]


def test_learned_selection_gain_low_precision_operands(oz):
    # the same batch with significands of bfloat16 / float16 / float32 /
    # float64 width: the network sees the narrow significands (its width
    # features) that the rule's mean-square statistic cannot, so the learned
    # start beats the rule in INT8 work and in time, and needs well under the
    # INT8 work of the smallest fixed s that passes every problem.  (That
    # fixed s, known here only after the fact, runs without the statistics
    # pass and the residual check.)
    out = _selection_gain(oz, "lowprec")
    assert out["learned"]["int8_tops"] < out["rule"]["int8_tops"] < out["fixed"]["int8_tops"]
    assert out["learned"]["int8_tops"] < 0.7 * out["fixed"]["int8_tops"]
    assert out["learned"]["ms_min"] < out["rule"]["ms_min"]
    assert out["learned"]["ms_min"] < out["escalate"]["ms_min"]
