"""Benchmark: effective FP64 TFLOP/s of the emulated ZGEMM on one MI355X.

Workload: one complex double GEMM C = A*B, square n = 4096, operands with a
per-row power-of-two exponent in [-20, 20] shared by real and imaginary parts
(normal(0,1) entries), emulated with s = 6 balanced (round-to-nearest) INT8
slices -- the smallest slice count whose error is below 1e-12 on this data
(truncated digits need s = 7: --digits 0 --slices 7).  One step is one
oz_zgemm call: exponent scan, digit split of both operands, the INT8
slice-pair GEMM(s) with the fused FP64 epilogue; by default in the
3-real-product form (three real products, the last one's epilogue combining
them; --zmode 4: one real product over the two-row form).  Inputs are
resident in HBM before timing.  The line reports the measured error against
the native product and whether it meets the metric's 1e-12.

Printed: one JSON line with the effective rate (8 n^3 / time), the roofline of
the dominant kernel (the INT8 GEMM, HIP events on its own stream), the native
FP64-MFMA ZGEMM (torch complex128 matmul, rocBLAS) on the same GPU, and the
CPU oracle timed on a bounded sample of the same workload.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "effective FP64 TFLOP/s at ≤1e-12 rel err vs native FP64-MFMA GEMM, same GPU"
INT8_PEAK_TOPS = 5000.0   # MI355X dense INT8 MFMA, vendor figure
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "gemm_traffic.json")
GEMM_SRC = os.path.join(ROOT, "paper_2503_22875_amd", "csrc", "oz_gemm.hip")


def pairs(s):
    return s * (s + 1) // 2


def traffic_for(workload):
    """HBM bytes per GEMM launch from committed rocprofv3 counters, or None
    when absent or taken on another version of the GEMM kernel source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    rec = json.load(open(TRAFFIC_FILE))
    sha = hashlib.sha256(open(GEMM_SRC, "rb").read()).hexdigest()
    ent = rec.get(workload)
    if not ent or ent.get("gemm_source_sha256") != sha:
        return None
    return ent["bytes_per_launch"]


def cpu_info():
    """CPU model, logical CPU count and the size of this process's affinity set."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"cpu_model": model, "cpu_count": os.cpu_count(), "affinity": len(os.sched_getaffinity(0))}


def cpu_baseline(A, B, s, C_gpu, rows, zmode=4, balanced=False, C_native=None):
    """Oracle on the first `rows` rows of C: O4 (the step-by-step CPU
    emulation, timed: the reported rate; the GPU rows checked bit for bit
    against it); on the first min(rows, 128) rows also O2 (the double-double
    product, the accuracy reference) and O1 (plain FP64), both timed, and the
    GPU and native rows' scale-weighted errors against O2."""
    import oracle
    cplx = np.iscomplexobj(A)
    As = np.asfortranarray(A[:rows])
    t0 = time.perf_counter()
    if cplx and zmode == 3:
        ref = oracle.emu_zgemm3("N", "N", As, B, s, balanced=balanced)
    else:
        ref = oracle.emu_gemm("N", "N", As, B, s, balanced=balanced)
    t = time.perf_counter() - t0
    r2 = min(rows, 128)
    A2 = np.asfortranarray(A[:r2])
    t1 = time.perf_counter()
    dd = oracle.gemm_dd("N", "N", A2, B)
    t_dd = time.perf_counter() - t1
    t2 = time.perf_counter()
    oracle.gemm_plain("N", "N", A2, B)
    t_plain = time.perf_counter() - t2
    n, k = B.shape[1], A.shape[1]
    if cplx:
        wa = np.abs(np.concatenate([A2.real, A2.imag], axis=1)).max(1)
        wb = np.abs(np.concatenate([B.real, B.imag], axis=0)).max(0)
    else:
        wa, wb = np.abs(A2).max(1), np.abs(B).max(0)
    fl = (8.0 if cplx else 2.0) * rows * n * k
    out = {
        "value": fl / t / 1e12,
        "unit": "TFLOP/s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": "rows 0..%d of C (all %d columns), same inputs and s; %.1f s wall" % (rows - 1, n, t),
        "sample_bit_exact": bool(np.array_equal(C_gpu[:rows], ref)),
        "rel_err_vs_double_double": oracle.weighted_error(C_gpu[:r2], dd, wa, wb),
        "o2_o1_sample": "rows 0..%d of C (all %d columns)" % (r2 - 1, n),
        "o2_double_double_s": round(t_dd, 2),
        "o1_plain_s": round(t_plain, 2),
    }
    if C_native is not None:
        out["native_rel_err_vs_double_double"] = oracle.weighted_error(C_native[:r2], dd, wa, wb)
    out.update(cpu_info())
    return out


def bench_batch(args):
    """Batched workload: 512 square complex products, n_b = 32 * randint(1, 16),
    s = --slices (6) with --digits (balanced by default), one persistent GEMM
    launch per replay of a captured HIP graph."""
    import torch

    import paper_2503_22875_amd as oz
    import workloads

    s = args.slices
    if not 1 <= s <= 8:
        raise SystemExit("batch512: fixed slice counts 1..8")
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    problems = workloads.zgemm_batch(512, seed=0)
    dev = [(torch.from_numpy(A.ravel(order="F")).cuda(), torch.from_numpy(B.ravel(order="F")).cuda(),
            torch.zeros(A.shape[0] * B.shape[1], dtype=torch.complex128, device="cuda")) for A, B in problems]
    ns = [A.shape[0] for A, _ in problems]
    torch.cuda.synchronize()
    h = oz.oz_create(0)
    oz.oz_set_stream(h, stream.cuda_stream)
    oz.oz_load_tuning(h)
    cnt = len(problems)
    plan = oz.oz_gemm_batched_plan(h, 1, "N" * cnt, "N" * cnt, ns, ns, ns, [1.0] * cnt, [d[0] for d in dev], ns,
                                   [d[1] for d in dev], ns, [0.0] * cnt, [d[2] for d in dev], ns,
                                   p=oz.prec(s, digits=args.digits, kernel=args.kernel, zmode=args.zmode))
    launches, tiles, nbytes, _ = oz.oz_batch_info(plan, cnt)
    # dominant kernel: the persistent GEMM launch, timed with events around it
    oz.oz_timing_enable(h, True)
    for _ in range(args.warmup):
        oz.oz_batch_execute(plan)
    oz.oz_timing_read(h)
    for _ in range(args.steps):
        oz.oz_batch_execute(plan)
    split_ms, gemm_ms, calls = oz.oz_timing_read(h)
    oz.oz_timing_enable(h, False)
    # headline: graph replays
    for _ in range(args.warmup):
        oz.oz_batch_graph_launch(plan)
    stream.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        oz.oz_batch_graph_launch(plan)
    e1.record(stream)
    stream.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    flops = sum(8.0 * n ** 3 for n in ns)
    # INT8 work: three real n x n x n products (3-product form) or one
    # (2n) x n x (2n) product over the two-row form
    int8_ops = sum(pairs(s) * 2.0 * (3 * n ** 3 if args.zmode == 3 else (2 * n) * n * (2 * n)) for n in ns)
    gemm_avg = gemm_ms / calls
    achieved = int8_ops / (gemm_avg * 1e-3) / 1e12
    out = {
        "metric": METRIC, "value": round(flops / (ms * 1e-3) / 1e12, 3), "unit": "TFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int8", "data": "synthetic",
        "config": {"workload": "batched zgemm: 512 square problems n_b = 32*randint(1,16), s=%d%s, %s, graph replay"
                               % (s, " balanced digits" if args.digits else "",
                                  "3-product form" if args.zmode == 3 else "4-product form"),
                   "slices": s, "digits": "balanced" if args.digits else "truncated", "zmode": args.zmode,
                   "problems": cnt, "sum_n3": int(sum(n ** 3 for n in ns)), "gemm_launches": launches,
                   "tiles": tiles, "plan_device_bytes": nbytes},
        "roofline": {"bound": "mfma", "achieved": round(achieved, 2), "peak": INT8_PEAK_TOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / INT8_PEAK_TOPS, 4), "traffic": None,
                     "kernel": "gemm_persistent_3m_kernel" if args.zmode == 3 else "gemm_persistent_kernel",
                     "avg_ms": round(gemm_avg, 4),
                     "split_avg_ms": round(split_ms / calls, 4)},
    }
    if not args.no_native:
        tA = [torch.from_numpy(A).cuda() for A, _ in problems]
        tB = [torch.from_numpy(B).cuda() for _, B in problems]
        tC = [None] * cnt
        with torch.cuda.stream(stream):
            for i in range(cnt):
                tC[i] = tA[i] @ tB[i]
        stream.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=stream):
            for i in range(cnt):
                tC[i] = tA[i] @ tB[i]
        for _ in range(2):
            g.replay()
        torch.cuda.synchronize()
        e0.record(torch.cuda.current_stream())
        for _ in range(args.steps):
            g.replay()
        e1.record(torch.cuda.current_stream())
        torch.cuda.synchronize()
        nms = e0.elapsed_time(e1) / args.steps
        worst = 0.0
        for i in range(cnt):
            got = dev[i][2].cpu().numpy().reshape(ns[i], ns[i], order="F")
            nat = tC[i].cpu().numpy()
            worst = max(worst, float(np.linalg.norm(got - nat) / np.linalg.norm(nat)))
        out["native_fp64"] = {"tflops": round(flops / (nms * 1e-3) / 1e12, 3), "ms": round(nms, 4),
                              "kind": "512 torch complex128 matmuls (rocBLAS zgemm) in one captured graph"}
        out["rel_err_vs_native_max"] = worst
        out["meets_tolerance"] = bool(worst <= 1e-12)
        out["speedup_vs_native"] = round(nms / ms, 3)
    oz.oz_batch_destroy(plan)
    oz.oz_destroy(h)
    print(json.dumps(out), flush=True)


def mixed_batch_on_device(oz, h, count=512, seed=0, kind="mixed"):
    """A heterogeneous batch (workloads.zgemm_batch_mixed, or with kind
    "lowprec" workloads.zgemm_batch_lowprec) drawn on the GPU by the library's
    counter-based generator: per problem the real and imaginary parts of A and
    B come from the two instances of workloads.mixed_parts, interleaved into
    complex column-major buffers.  Returns (dev, ns, tols, params) with dev a
    list of (A, B, C) tensors."""
    import torch

    import workloads
    gen = workloads.zgemm_batch_lowprec if kind == "lowprec" else workloads.zgemm_batch_mixed
    params, tols = gen(count, seed)
    dev, ns = [], []
    for p in params:
        n = p["n"]
        parts = []
        for q in workloads.mixed_parts(p):
            A = torch.empty(n * n, dtype=torch.float64, device="cuda")
            B = torch.empty(n * n, dtype=torch.float64, device="cuda")
            oz.oz_gen_operands(h, q, A, n, B, n)
            parts.append((A, B))
        torch.cuda.synchronize()
        # imaginary parts: scaled by the real parts' per-vector powers of two (exact)
        ea, eb = workloads.vector_exponents(p)
        sa = torch.pow(2.0, torch.from_numpy(ea).double()).cuda()
        sb = torch.pow(2.0, torch.from_numpy(eb).double()).cuda()
        Ai = (parts[1][0].view(n, n) * sa[None, :]).reshape(-1)  # storage view [column][row]
        Bi = (parts[1][1].view(n, n) * sb[:, None]).reshape(-1)
        parts[1] = (Ai, Bi)
        Az = torch.view_as_complex(torch.stack([parts[0][0], parts[1][0]], dim=1).contiguous())
        Bz = torch.view_as_complex(torch.stack([parts[0][1], parts[1][1]], dim=1).contiguous())
        dev.append((Az, Bz, torch.zeros(n * n, dtype=torch.complex128, device="cuda")))
        ns.append(n)
    return dev, ns, tols, params


def selection_gain(oz, h, stream, dev, ns, tols, steps=5, warmup=2, fixed_max=12):
    """Time and accuracy of one tolerance-driven batch run four ways, with
    per-problem tolerances tols[i]:
      fixed:    one slice count for every problem, the smallest s at which
                every problem meets its tolerance by its true error (found by
                trying s = 1, 2, ...; known only after the fact), run as a
                plain fixed plan (s <= 8) or a tolerance plan pinned at s;
      rule:     starting s per problem from the operand-statistics rule,
                residual check and growth;
      escalate: every problem starts at s = 2, check and growth;
      learned:  starting s per problem from the trained network, check and
                growth.
    True error = scale-weighted error against the emulation at s = 12 (the
    fixed-s emulation as judge; its own error is about 2^-84).  Time = whole
    execution on the stream, median (and min) of `steps` runs after `warmup`.
    Returns a dict of rows."""
    import torch

    cnt = len(ns)
    tols = np.asarray(tols, dtype=np.float64)
    pairs_ops = lambda s, n: s * (s + 1) // 2 * 2.0 * (2 * n) * n * (2 * n)  # INT8 ops, 4-product form
    # judge: the s = 12 emulation of every problem, and the scale weights
    ref, wts = [], []
    for (dA, dB, _), n in zip(dev, ns):
        Cr = torch.zeros(n * n, dtype=torch.complex128, device="cuda")
        oz.oz_zgemm(h, "N", "N", n, n, n, 1.0, dA, n, dB, n, 0.0, Cr, n, oz.prec(12))
        ref.append(Cr.view(n, n))
        Ad, Bd = dA.view(n, n).t(), dB.view(n, n).t()  # row-major views of column-major storage
        wa = torch.maximum(Ad.real.abs(), Ad.imag.abs()).amax(1)
        wb = torch.maximum(Bd.real.abs(), Bd.imag.abs()).amax(0)
        wa = torch.where(wa > 0, 1.0 / wa, torch.zeros_like(wa))
        wb = torch.where(wb > 0, 1.0 / wb, torch.zeros_like(wb))
        wts.append((wb[:, None] * wa[None, :]))  # transposed like the storage views
    torch.cuda.synchronize()

    def true_errors():
        errs = []
        for (_, _, dC), n, Cr, W in zip(dev, ns, ref, wts):
            C = dC.view(n, n)
            den = torch.linalg.norm(W * Cr)
            num = torch.linalg.norm(W * (C - Cr))
            errs.append(float(num / den) if float(den) > 0 else float(num))
        return np.array(errs)

    def run(p, per_problem_tols):
        plan = oz.oz_gemm_batched_plan(h, 1, "N" * cnt, "N" * cnt, ns, ns, ns, [1.0] * cnt, [d[0] for d in dev], ns,
                                       [d[1] for d in dev], ns, [0.0] * cnt, [d[2] for d in dev], ns, p=p,
                                       tols=per_problem_tols)
        try:
            for _ in range(warmup):
                oz.oz_batch_execute(plan)
            stream.synchronize()
            times = []
            for _ in range(steps):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                oz.oz_batch_execute(plan)
                e1.record(stream)
                stream.synchronize()
                times.append(e0.elapsed_time(e1))
            reps = oz.oz_batch_report(plan, cnt)
        finally:
            oz.oz_batch_destroy(plan)
        err = true_errors()
        final = np.array([r.slices_used for r in reps])
        start = final - np.array([r.fallbacks for r in reps])
        return {"ms": round(float(np.median(times)), 3), "ms_min": round(float(np.min(times)), 3),
                "mean_start": round(float(start.mean()), 3), "mean_final": round(float(final.mean()), 3),
                "grown": int((final > start).sum()),
                "int8_tops": round(sum(pairs_ops(int(s), n) for s, n in zip(final, ns)) / 1e12, 3),
                "pass_true": float(np.mean(err <= tols)), "worst_err_over_tol": float(np.max(err / tols))}

    out = {}
    tl = [float(t) for t in tols]
    # fixed: the smallest single s that passes every problem
    for s in range(1, fixed_max + 1):
        if s <= 8:
            row = run(oz.prec(s), None)
        else:
            row = run(oz.prec(0, tol=1.0, smax=s, sstart=s), tl)
        if row["pass_true"] == 1.0:
            row["s"] = s
            out["fixed"] = row
            break
    out["rule"] = run(oz.prec(0, tol=1.0, smax=12, selector=0), tl)
    out["escalate"] = run(oz.prec(0, tol=1.0, smax=12, sstart=2), tl)
    out["learned"] = run(oz.prec(0, tol=1.0, smax=12, selector=1), tl)
    if "fixed" in out:
        out["learned_speedup"] = {k: round(out[k]["ms"] / out["learned"]["ms"], 3)
                                  for k in ("fixed", "rule", "escalate")}
    return out


def bench_select(args):
    """Gain of the learned slice-count selector on tolerance-driven batches of
    512 square complex problems (n_b = 32 * randint(1, 16)), each run as
    fixed / rule / escalate / learned (``selection_gain``):
      normal: the batched workload (N(0,1) entries) at one tolerance for the
              batch, tol in --select-tols;
      mixed:  the heterogeneous batch (workloads.zgemm_batch_mixed, drawn on
              the GPU): every problem with its own structure from the
              selector's instance distribution and its own tolerance,
              log-uniform in [1e-15, 1e-4];
      lowprec: the same with significands of bfloat16 / float16 / float32 /
              float64 width (workloads.zgemm_batch_lowprec)."""
    import torch

    import paper_2503_22875_amd as oz
    import workloads

    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    h = oz.oz_create(0)
    oz.oz_set_stream(h, stream.cuda_stream)
    oz.oz_load_tuning(h)
    if not os.path.exists(oz.SELECTOR_PATH):
        raise SystemExit("no trained selector at %s (python -m paper_2503_22875_amd.train_selector)" %
                         oz.SELECTOR_PATH)
    net = oz.oz_mlp_load(h)
    oz.oz_set_selector(h, net)
    results = []
    for dname in args.select_data.split(","):
        if dname in ("mixed", "lowprec"):
            dev, ns, tols, _ = mixed_batch_on_device(oz, h, 512, seed=0, kind=dname)
            cases = [("own", tols)]
        else:
            problems = workloads.zgemm_batch(512, seed=0)
            ns = [A.shape[0] for A, _ in problems]
            dev = [(torch.from_numpy(A.ravel(order="F")).cuda(), torch.from_numpy(B.ravel(order="F")).cuda(),
                    torch.zeros(A.shape[0] * B.shape[1], dtype=torch.complex128, device="cuda"))
                   for A, B in problems]
            del problems
            cases = [(t, [float(t)] * len(ns)) for t in args.select_tols.split(",")]
        torch.cuda.synchronize()
        flops = sum(8.0 * n ** 3 for n in ns)
        for tname, tl in cases:
            print("select: data %s, tol %s" % (dname, tname), flush=True)
            row = {"data": dname, "tol": tname}
            row.update(selection_gain(oz, h, stream, dev, ns, tl, steps=args.steps, warmup=args.warmup))
            for k in ("fixed", "rule", "escalate", "learned"):
                if k in row:
                    row[k]["tflops"] = round(flops / (row[k]["ms"] * 1e-3) / 1e12, 2)
            print(json.dumps(row), flush=True)
            results.append(row)
        del dev
        torch.cuda.empty_cache()
    oz.oz_set_selector(h, None)
    oz.oz_mlp_destroy(net)
    oz.oz_destroy(h)
    print(json.dumps({"workload": "selector gain", "rows": results}), flush=True)


def _time_ms(fn, stream, steps, warmup):
    """Mean milliseconds per call of fn() on `stream` (HIP events)."""
    import torch
    for _ in range(warmup):
        fn()
    stream.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    stream.synchronize()
    return e0.elapsed_time(e1) / steps


def _weighted_err(C, Cn, wa, wb):
    """Scale-weighted relative error of C against Cn (torch tensors on the GPU)."""
    import torch
    W = (1.0 / wa)[:, None] * (1.0 / wb)[None, :]
    return float(torch.linalg.norm(W * (C - Cn)) / torch.linalg.norm(W * Cn))


def bench_sweep(args):
    """Slice-count sweep of the square ZGEMM (row exponents in [-20, 20]):
    n = 2048 and 4096, s = 3 .. 8, both complex forms.  Per point: time per
    call, effective FP64 rate, and the scale-weighted error against the
    native complex128 product (rocBLAS zgemm on the same GPU, timed beside)."""
    import torch

    import paper_2503_22875_amd as oz
    import workloads

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    h = oz.oz_create(0)
    oz.oz_set_stream(h, stream.cuda_stream)
    rows = []
    for n in [int(v) for v in args.sweep_n.split(",")]:
        A, B = workloads.zgemm_rowexp(n, seed=0)
        dA = torch.from_numpy(A.ravel(order="F")).cuda()
        dB = torch.from_numpy(B.ravel(order="F")).cuda()
        dC = torch.zeros(n * n, dtype=torch.complex128, device="cuda")
        tA, tB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
        del A, B
        out = {}
        nms = _time_ms(lambda: out.__setitem__("C", tA @ tB), stream, args.steps, 3)
        Cn = out["C"]
        wa = torch.maximum(tA.real.abs(), tA.imag.abs()).amax(1)
        wb = torch.maximum(tB.real.abs(), tB.imag.abs()).amax(0)
        flops = 8.0 * n ** 3
        for zmode in (3, 4):
            for s in range(3, 9):
                p = oz.prec(s, zmode=zmode)
                ms = _time_ms(lambda: oz.oz_zgemm(h, "N", "N", n, n, n, 1.0, dA, n, dB, n, 0.0, dC, n, p),
                              stream, args.steps, args.warmup)
                C = dC.view(n, n).t()
                row = {"n": n, "zmode": zmode, "s": s, "ms": round(ms, 4),
                       "tflops": round(flops / (ms * 1e-3) / 1e12, 2),
                       "speedup_vs_native": round(nms / ms, 3),
                       "err_vs_native": _weighted_err(C, Cn, wa, wb)}
                print(json.dumps(row), flush=True)
                rows.append(row)
        rows.append({"n": n, "native_ms": round(nms, 4), "native_tflops": round(flops / (nms * 1e-3) / 1e12, 2)})
        print(json.dumps(rows[-1]), flush=True)
        del dA, dB, dC, tA, tB, Cn
        torch.cuda.empty_cache()
    oz.oz_destroy(h)
    print(json.dumps({"workload": "zgemm slice sweep (row exponents +-20, normal entries)", "rows": rows}),
          flush=True)


def bench_wide_tol(args):
    """Tolerance-driven wide-range DGEMM: m = n = 4096, k = 8192, rows of A and
    columns of B scaled by 10^U(-8, 8), tol 1e-6, 1e-10, 1e-14 (smax 12;
    --wide-digits 1: balanced digits, smax 8).
    Per tolerance: time of the whole call (selection, split, products, checks,
    growth), the start and final slice counts, the check's estimate, the true
    scale-weighted error against the native float64 product, and the time of
    a fixed-s call at the final s (no check) and of the native DGEMM."""
    import torch

    import paper_2503_22875_amd as oz
    import workloads

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    h = oz.oz_create(0)
    oz.oz_set_stream(h, stream.cuda_stream)
    m, n, k = 4096, 4096, 8192
    A, B = workloads.dgemm_wide(m, n, k, seed=0)
    dA = torch.from_numpy(A.ravel(order="F")).cuda()
    dB = torch.from_numpy(B.ravel(order="F")).cuda()
    dC = torch.zeros(m * n, dtype=torch.float64, device="cuda")
    tA, tB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    del A, B
    out = {}
    nms = _time_ms(lambda: out.__setitem__("C", tA @ tB), stream, args.steps, 3)
    Cn = out["C"]
    wa, wb = tA.abs().amax(1), tB.abs().amax(0)
    flops = 2.0 * m * n * k
    rows = []
    dig = args.wide_digits
    for tol in [float(v) for v in args.wide_tols.split(",")]:
        p = oz.prec(0, tol=tol, smax=12, digits=dig)
        ms = _time_ms(lambda: oz.oz_dgemm(h, "N", "N", m, n, k, 1.0, dA, m, dB, k, 0.0, dC, m, p),
                      stream, args.steps, args.warmup)
        st, rep = oz.oz_dgemm(h, "N", "N", m, n, k, 1.0, dA, m, dB, k, 0.0, dC, m, p, report=True)
        C = dC.view(n, m).t()
        err = _weighted_err(C, Cn, wa, wb)
        s1 = rep.slices_used
        pf = oz.prec(s1, digits=dig) if s1 <= 8 else oz.prec(0, tol=tol, smax=s1, sstart=s1)
        fms = _time_ms(lambda: oz.oz_dgemm(h, "N", "N", m, n, k, 1.0, dA, m, dB, k, 0.0, dC, m, pf),
                       stream, args.steps, args.warmup)
        row = {"tol": tol, "ms": round(ms, 4), "tflops": round(flops / (ms * 1e-3) / 1e12, 2),
               "speedup_vs_native": round(nms / ms, 3), "start_s": s1 - rep.fallbacks, "final_s": s1,
               "estimate": rep.resid_est, "err_vs_native": err, "met": bool(err <= tol),
               "fixed_s_ms": round(fms, 4), "fixed_s_tflops": round(flops / (fms * 1e-3) / 1e12, 2)}
        print(json.dumps(row), flush=True)
        rows.append(row)
    oz.oz_destroy(h)
    print(json.dumps({"workload": "wide-range dgemm 4096x4096x8192 (rows/cols x 10^U(-8,8)), tolerance-driven, %s digits"
                      % ("balanced" if dig else "truncated"),
                      "native_ms": round(nms, 4), "native_tflops": round(flops / (nms * 1e-3) / 1e12, 2),
                      "rows": rows}), flush=True)


def bench_dgemm(args):
    """Real DGEMM C = A*B, m = n = k = --n (4096), entries U(-1, 1) * 2^randint(-4, 4)
    (the 256^3 case's recipe at full size), emulated with --slices (6) and
    --digits (balanced): the smallest configuration whose scale-weighted error
    against the double-double product is below 1e-12 on this data (balanced
    s = 5: 4.8e-11, truncated s = 6: 6.5e-12, truncated s = 7: 6e-14).  Same
    report as the ZGEMM line: effective rate 2 n^3 / time, the GEMM kernel's
    roofline, native float64 matmul (rocBLAS dgemm) with its error, and the
    oracle on a sample of rows."""
    import torch

    import paper_2503_22875_amd as oz
    import workloads

    n, s = args.n, args.slices
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    A, B = workloads.dgemm_uniform(n, n, n, seed=0)
    dA = torch.from_numpy(A.ravel(order="F")).cuda()
    dB = torch.from_numpy(B.ravel(order="F")).cuda()
    dC = torch.zeros(n * n, dtype=torch.float64, device="cuda")
    h = oz.oz_create(0)
    oz.oz_set_stream(h, stream.cuda_stream)
    p = oz.prec(s, kernel=args.kernel, digits=args.digits)

    def step():
        oz.oz_dgemm(h, "N", "N", n, n, n, 1.0, dA, n, dB, n, 0.0, dC, n, p)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    oz.oz_timing_enable(h, True)
    oz.oz_timing_read(h)
    ms = _time_ms(step, stream, args.steps, 0)
    split_ms, gemm_ms, calls = oz.oz_timing_read(h)
    oz.oz_timing_enable(h, False)
    flops = 2.0 * n ** 3
    int8_ops = pairs(s) * 2.0 * n ** 3
    gemm_avg_ms = gemm_ms / calls
    achieved = int8_ops / (gemm_avg_ms * 1e-3) / 1e12
    C_gpu = dC.cpu().numpy().reshape(n, n, order="F")
    digits = "balanced digits" if args.digits == 1 else "truncated digits"
    out = {"metric": METRIC, "workload": "dgemm n=%d s=%d %s (entries U(-1,1) * 2^randint(-4,4))" % (n, s, digits),
           "ms": round(ms, 4), "tflops": round(flops / (ms * 1e-3) / 1e12, 3),
           "roofline": {"bound": "mfma", "achieved": round(achieved, 2), "peak": INT8_PEAK_TOPS, "unit": "TFLOP/s",
                        "frac": round(achieved / INT8_PEAK_TOPS, 4), "avg_ms": round(gemm_avg_ms, 4),
                        "split_avg_ms": round(split_ms / calls, 4)}}
    tA, tB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    res = {}
    nms = _time_ms(lambda: res.__setitem__("C", tA @ tB), stream, args.steps, 3)
    Cn = res["C"].cpu().numpy()
    out["native_fp64"] = {"tflops": round(flops / (nms * 1e-3) / 1e12, 3), "ms": round(nms, 4),
                          "kind": "torch float64 matmul (rocBLAS dgemm)"}
    out["speedup_vs_native"] = round(nms / ms, 3)
    if not args.no_cpu:
        cb = cpu_baseline(A, B, s, C_gpu, args.cpu_rows, balanced=args.digits == 1, C_native=Cn)
        out["cpu_baseline"] = cb
        out["meets_tolerance"] = bool(cb["rel_err_vs_double_double"] <= 1e-12)
    oz.oz_destroy(h)
    print(json.dumps(out), flush=True)


def bench_peaks(args):
    """The rates the roofline fractions divide by, measured by the library's
    own microbenchmarks (oz_peak): INT8 MFMA (v_mfma_i32_32x32x32_i8, the
    slice GEMM's shape, with fixed small operands and with full-range operands
    that change between instructions, and v_mfma_i32_16x16x64_i8), FP64 MFMA
    (v_mfma_f64_16x16x4_f64) and a 1 GiB device copy; best of --steps."""
    import torch

    import paper_2503_22875_amd as oz

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    h = oz.oz_create(0)
    oz.oz_set_stream(h, stream.cuda_stream)
    src = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    i8 = max(oz.oz_peak(h, 0, 20000) for _ in range(args.steps))
    i8_16 = max(oz.oz_peak(h, 3, 20000) for _ in range(args.steps))
    i8_rand = max(oz.oz_peak(h, 4, 20000) for _ in range(args.steps))
    f64 = max(oz.oz_peak(h, 1, 20000) for _ in range(args.steps))
    cp = max(oz.oz_peak(h, 2, 10, src, dst, src.numel() * 8) for _ in range(args.steps))
    oz.oz_destroy(h)
    print(json.dumps({"workload": "peaks", "int8_mfma_tops": round(i8 / 1e12, 1),
                      "int8_mfma_16x16x64_tops": round(i8_16 / 1e12, 1),
                      "int8_mfma_random_operands_tops": round(i8_rand / 1e12, 1),
                      "int8_vendor_tops": INT8_PEAK_TOPS, "fp64_mfma_tflops": round(f64 / 1e12, 2),
                      "fp64_vendor_tflops": 78.6, "copy_gbs": round(cp / 1e9, 1), "hbm_vendor_gbs": 8000.0,
                      "copy_bytes": src.numel() * 8}), flush=True)


def bench_blas(args):
    """The BLAS offload layer on host arrays: zgemm_ (n = 4096, s = 7, the
    3-product form) through liboz_blas.so, timed by wall clock per call with
    the PCIe copies of A, B and C included, beside the same layer in native
    FP64 mode (rocBLAS zgemm with the same copies).  The split of each call
    into copy and product time comes from the layer's own event counters."""
    os.environ.setdefault("OZ_ZMODE", "3")
    import paper_2503_22875_amd.blas as blas
    import workloads

    n = 4096
    A, B = workloads.zgemm_rowexp(n, seed=0)
    C = np.zeros((n, n), np.complex128, order="F")
    flops = 8.0 * n ** 3
    rows = []
    for mode in ("fp64_int8_7", "dgemm"):
        assert blas.oz_blas_set_mode(mode)
        for _ in range(2):
            blas.zgemm_("N", "N", n, n, n, 1.0, A, n, B, n, 0.0, C, n)
        s0 = blas.oz_blas_stats()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            blas.zgemm_("N", "N", n, n, n, 1.0, A, n, B, n, 0.0, C, n)
        wall = (time.perf_counter() - t0) * 1e3 / args.steps
        s1 = blas.oz_blas_stats()
        calls = s1.calls - s0.calls
        copy_ms = (s1.copy_ms - s0.copy_ms) / calls
        comp_ms = (s1.compute_ms - s0.compute_ms) / calls
        row = {"mode": mode, "wall_ms": round(wall, 3), "tflops_pcie_inclusive": round(flops / (wall * 1e-3) / 1e12, 2),
               "copy_ms": round(copy_ms, 3), "product_ms": round(comp_ms, 3),
               "tflops_product_only": round(flops / (comp_ms * 1e-3) / 1e12, 2),
               "bytes_per_call": int((s1.bytes_to_device - s0.bytes_to_device + s1.bytes_to_host - s0.bytes_to_host)
                                     / calls)}
        print(json.dumps(row), flush=True)
        rows.append(row)
    blas.oz_blas_finalize()
    print(json.dumps({"workload": "zgemm_ n=4096 s=7 3-product form from host arrays (PCIe copies included)",
                      "rows": rows}), flush=True)


def bench_x2(args):
    """Products beyond FP64: DGEMM n = 4096 (N(0,1) entries) with a
    double-double result (oz_dgemm_x2) at s = 8, 10, 12, 14, beside the FP64
    result at the same s (oz_dgemm, default kernel) and the per-diagonal
    streaming kernel (kernel 3).  The accuracy of the double-double result is
    checked by the GPU tests against the exact product; this line reports time
    only."""
    import torch

    import paper_2503_22875_amd as oz

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    h = oz.oz_create(0)
    oz.oz_set_stream(h, stream.cuda_stream)
    n = 4096
    rng = np.random.default_rng(0)
    dA = torch.from_numpy(rng.standard_normal(n * n)).cuda()
    dB = torch.from_numpy(rng.standard_normal(n * n)).cuda()
    dH = torch.zeros(n * n, dtype=torch.float64, device="cuda")
    dL = torch.zeros(n * n, dtype=torch.float64, device="cuda")
    flops = 2.0 * n ** 3
    rows = []
    for s in (8, 10, 12, 14):
        p = oz.prec(s)
        ps = oz.prec(s, kernel=3)
        ms_x2 = _time_ms(lambda: oz.oz_dgemm_x2(h, "N", "N", n, n, n, dA, n, dB, n, dH, dL, n, p), stream,
                         args.steps, args.warmup)
        ms_d = _time_ms(lambda: oz.oz_dgemm(h, "N", "N", n, n, n, 1.0, dA, n, dB, n, 0.0, dH, n, p), stream,
                        args.steps, args.warmup)
        ms_s = _time_ms(lambda: oz.oz_dgemm(h, "N", "N", n, n, n, 1.0, dA, n, dB, n, 0.0, dH, n, ps), stream,
                        args.steps, args.warmup)
        row = {"s": s, "x2_ms": round(ms_x2, 3), "x2_tflops": round(flops / (ms_x2 * 1e-3) / 1e12, 2),
               "fp64_ms": round(ms_d, 3), "fp64_tflops": round(flops / (ms_d * 1e-3) / 1e12, 2),
               "streaming_ms": round(ms_s, 3), "streaming_tflops": round(flops / (ms_s * 1e-3) / 1e12, 2)}
        print(json.dumps(row), flush=True)
        rows.append(row)
    oz.oz_destroy(h)
    print(json.dumps({"workload": "dgemm n=4096 double-double result", "rows": rows}), flush=True)


def bench_inv(args):
    """LU-based complex inversion, n = 4096 (entries N(0,1) + i N(0,1)): time
    of oz_zgetrf + oz_zgetri at s = 3..8 and 14 (panel width nb, solve blocks
    nb_inv), beside the
    native FP64 inverse (torch.linalg.inv, same GPU).  Per s: the inverse's
    largest entry error relative to the largest entry of the native inverse,
    its residual max |A X - I|, and the effective rate on LAPACK's operation
    count of getrf + getri (8 n^3 real flops for complex).  Then the same with
    every product tolerance-driven (each picks its own s) at --inv-tols."""
    import torch

    import paper_2503_22875_amd as oz
    import workloads

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    h = oz.oz_create(0)
    oz.oz_set_stream(h, stream.cuda_stream)
    n, nb, nbi = args.n, args.nb, args.nb_inv
    A = workloads.zinv_gauss(n, seed=0)
    Ad = torch.from_numpy(A).cuda()
    dA0 = torch.view_as_real(torch.from_numpy(np.ascontiguousarray(A.T))).reshape(-1).cuda()
    dA = torch.empty_like(dA0)
    dX = torch.empty_like(dA0)
    ipiv = torch.empty(n, dtype=torch.int32, device="cuda")
    eye = torch.eye(n, dtype=torch.complex128, device="cuda")
    flops = 8.0 * n ** 3
    steps = max(1, min(args.steps, 5))
    ms_nat = _time_ms(lambda: torch.linalg.inv(Ad), stream, steps, 1)
    Xr = torch.linalg.inv(Ad)
    resid_nat = float((Ad @ Xr - eye).abs().max())
    rows = []
    for s in [int(v) for v in args.inv_slices.split(",")]:
        p = oz.prec(s)

        def run():
            dA.copy_(dA0)
            oz.oz_zgetrf(h, n, dA, n, ipiv, nb, p)
            oz.oz_zgetri(h, n, dA, n, ipiv, dX, n, nbi, p)

        run()
        X = torch.view_as_complex(dX.view(n, n, 2)).T
        err = float((X - Xr).abs().max() / Xr.abs().max())
        resid = float((Ad @ X - eye).abs().max())
        ms = _time_ms(run, stream, steps, 1)
        row = {"s": s, "ms": round(ms, 3), "tflops_eff": round(flops / (ms * 1e-3) / 1e12, 2),
               "err_vs_native": float("%.3e" % err), "resid": float("%.3e" % resid)}
        print(json.dumps(row), flush=True)
        rows.append(row)
    for s in [int(v) for v in args.inv_balanced.split(",") if v]:
        p = oz.prec(s, digits=1)

        def run_bal():
            dA.copy_(dA0)
            oz.oz_zgetrf(h, n, dA, n, ipiv, nb, p)
            oz.oz_zgetri(h, n, dA, n, ipiv, dX, n, nbi, p)

        run_bal()
        X = torch.view_as_complex(dX.view(n, n, 2)).T
        err = float((X - Xr).abs().max() / Xr.abs().max())
        resid = float((Ad @ X - eye).abs().max())
        ms = _time_ms(run_bal, stream, steps, 1)
        row = {"s": s, "digits": "balanced", "ms": round(ms, 3), "tflops_eff": round(flops / (ms * 1e-3) / 1e12, 2),
               "err_vs_native": float("%.3e" % err), "resid": float("%.3e" % resid)}
        print(json.dumps(row), flush=True)
        rows.append(row)
    for tol in [float(v) for v in args.inv_tols.split(",") if v]:
        p = oz.prec(0, tol=tol)

        def run_tol():
            dA.copy_(dA0)
            oz.oz_zgetrf(h, n, dA, n, ipiv, nb, p)
            oz.oz_zgetri(h, n, dA, n, ipiv, dX, n, nbi, p)

        run_tol()
        X = torch.view_as_complex(dX.view(n, n, 2)).T
        err = float((X - Xr).abs().max() / Xr.abs().max())
        resid = float((Ad @ X - eye).abs().max())
        ms = _time_ms(run_tol, stream, steps, 1)
        row = {"tol": tol, "ms": round(ms, 3), "tflops_eff": round(flops / (ms * 1e-3) / 1e12, 2),
               "err_vs_native": float("%.3e" % err), "resid": float("%.3e" % resid)}
        print(json.dumps(row), flush=True)
        rows.append(row)
    oz.oz_destroy(h)
    print(json.dumps({"workload": "complex LU inversion n=%d nb=%d/%d (N(0,1)+iN(0,1))" % (n, nb, nbi),
                      "native": {"ms": round(ms_nat, 3), "tflops_eff": round(flops / (ms_nat * 1e-3) / 1e12, 2),
                                 "resid": float("%.3e" % resid_nat)},
                      "rows": rows}), flush=True)


def bench_balanced(args):
    """Truncated vs balanced (round-to-nearest) digits: ZGEMM n = 4096 (row
    exponents +-20, normal entries) in the 4-product and the 3-product form at
    s = 3..8, each with its time per call and relative error (Frobenius)
    against the native complex128 product on the same GPU."""
    import torch

    import paper_2503_22875_amd as oz
    import workloads

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    h = oz.oz_create(0)
    oz.oz_set_stream(h, stream.cuda_stream)
    n = args.n
    A, B = workloads.zgemm_rowexp(n, seed=0)
    Ad = torch.from_numpy(A).cuda()
    Bd = torch.from_numpy(B).cuda()
    dA = torch.view_as_real(Ad.T.contiguous()).reshape(-1)
    dB = torch.view_as_real(Bd.T.contiguous()).reshape(-1)
    dC = torch.empty_like(dA)
    N = Ad @ Bd
    nrm = float(torch.linalg.norm(N))
    flops = 8.0 * n ** 3
    rows = []
    for zmode, s in [(z, s) for z in (4, 3) for s in range(3, 9)]:
        row = {"s": s, "zmode": zmode}
        for name, dig in (("truncated", 0), ("balanced", 1)):
            p = oz.prec(s, digits=dig, zmode=zmode)
            ms = _time_ms(lambda: oz.oz_zgemm(h, "N", "N", n, n, n, 1.0, dA, n, dB, n, 0.0, dC, n, p), stream,
                          args.steps, args.warmup)
            C = torch.view_as_complex(dC.view(n, n, 2)).T
            err = float(torch.linalg.norm(C - N)) / nrm
            row[name] = {"ms": round(ms, 3), "tflops": round(flops / (ms * 1e-3) / 1e12, 2),
                         "rel_err_vs_native": float("%.3e" % err)}
        print(json.dumps(row), flush=True)
        rows.append(row)
    oz.oz_destroy(h)
    print(json.dumps({"workload": "zgemm n=%d, truncated vs balanced digits" % n, "rows": rows}),
          flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="zgemm4096",
                    choices=["zgemm4096", "dgemm", "peaks", "batch512", "select", "sweep", "wide_tol", "blas", "x2",
                             "inv", "balanced"])
    ap.add_argument("--nb", type=int, default=128, help="panel width of the inversion workload (getrf)")
    ap.add_argument("--nb-inv", type=int, default=256, help="block rows of the inversion workload's solves (getri)")
    ap.add_argument("--inv-slices", default="3,4,5,6,7,8,14")
    ap.add_argument("--inv-balanced", default="4,5,6,7",
                    help="inversion rows with balanced digits in every product (slice counts)")
    ap.add_argument("--inv-tols", default="1e-8,1e-10,1e-12",
                    help="tolerance-driven rows of the inversion workload (each product picks its own s)")
    ap.add_argument("--select-data", default="mixed,lowprec,normal")
    ap.add_argument("--select-tols", default="1e-10,1e-12,1e-14")
    ap.add_argument("--sweep-n", default="2048,4096")
    ap.add_argument("--wide-tols", default="1e-6,1e-10,1e-12,1e-14")
    ap.add_argument("--wide-digits", type=int, default=0, choices=[0, 1],
                    help="wide_tol workload: 1 = balanced digits (smax 8)")
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--slices", type=int, default=6)
    ap.add_argument("--digits", type=int, default=1, choices=[0, 1],
                    help="1 = balanced (round-to-nearest) digits (default), 0 = truncated digits")
    ap.add_argument("--zmode", type=int, default=None, choices=[0, 3, 4],
                    help="complex form: 3 = three real products, 4 = one real product over the two-row form, "
                         "0 = the library's choice (default: 3 for single ZGEMM workloads, 0 for batches)")
    ap.add_argument("--kernel", type=int, default=0, choices=[0, 1, 2, 4, 5],
                    help="GEMM kernel shape (as oz_prec_t.kernel; 0 = the default shape)")
    ap.add_argument("--cpu-rows", type=int, default=512)
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one plain 1 GiB device copy (reference for HBM byte counters)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-native", action="store_true")
    args = ap.parse_args()
    if args.zmode is None:
        # batches: the library's choice (the 4-product form, measured faster
        # there); single ZGEMM workloads: the 3-product form
        args.zmode = 0 if args.workload in ("batch512", "select") else 3
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.workload == "dgemm":
        return bench_dgemm(args)
    if args.workload == "peaks":
        return bench_peaks(args)
    if args.workload == "batch512":
        return bench_batch(args)
    if args.workload == "select":
        return bench_select(args)
    if args.workload == "sweep":
        return bench_sweep(args)
    if args.workload == "wide_tol":
        return bench_wide_tol(args)
    if args.workload == "blas":
        return bench_blas(args)
    if args.workload == "x2":
        return bench_x2(args)
    if args.workload == "inv":
        return bench_inv(args)
    if args.workload == "balanced":
        return bench_balanced(args)

    import torch

    import paper_2503_22875_amd as oz
    import workloads

    n, s = args.n, args.slices
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    A, B = workloads.zgemm_rowexp(n, seed=0)
    dA = torch.from_numpy(A.ravel(order="F")).cuda()
    dB = torch.from_numpy(B.ravel(order="F")).cuda()
    dC = torch.zeros(n * n, dtype=torch.complex128, device="cuda")
    h = oz.oz_create(0)
    oz.oz_set_stream(h, stream.cuda_stream)
    p = oz.prec(s, zmode=args.zmode, kernel=args.kernel, digits=args.digits)

    def step():
        oz.oz_zgemm(h, "N", "N", n, n, n, 1.0, dA, n, dB, n, 0.0, dC, n, p)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    oz.oz_timing_enable(h, True)
    oz.oz_timing_read(h)
    t0.record(stream)
    for _ in range(args.steps):
        step()
    t1.record(stream)
    torch.cuda.synchronize()
    split_ms, gemm_ms, calls = oz.oz_timing_read(h)
    oz.oz_timing_enable(h, False)
    ms = t0.elapsed_time(t1) / args.steps
    # per-call spread (a second pass, one event pair per call)
    per_call = []
    for _ in range(args.steps):
        c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        c0.record(stream)
        step()
        c1.record(stream)
        c1.synchronize()
        per_call.append(c0.elapsed_time(c1))
    flops = 8.0 * n ** 3
    value = flops / (ms * 1e-3) / 1e12

    C_gpu = dC.cpu().numpy().reshape(n, n, order="F")

    # dominant kernel: the INT8 slice GEMM, P(s) pairs; 4-product form: one
    # launch over C' = A' B' (2n x n x 2n); 3-product form: three n x n x n
    # launches (the timed GEMM phase spans all three)
    launches = 3 if args.zmode == 3 else 1
    int8_ops = pairs(s) * 2.0 * ((2 * n) * n * (2 * n) if args.zmode != 3 else n * n * n)
    gemm_avg_ms = gemm_ms / calls / launches
    achieved = int8_ops / (gemm_avg_ms * 1e-3) / 1e12
    form = "3-product form" if args.zmode == 3 else "4-product form"
    digits = "balanced digits" if args.digits == 1 else "truncated digits"
    workload = "zgemm n=%d s=%d %s (row exponents +-20, normal entries)" % (n, s, form)
    if args.digits == 1:
        workload = "zgemm n=%d s=%d %s, balanced digits (row exponents +-20, normal entries)" % (n, s, form)
    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "ms_per_call": {"median": round(float(np.median(per_call)), 4), "min": round(float(np.min(per_call)), 4)},
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int8",
        "data": "synthetic",
        "config": {"workload": workload, "m": n, "n": n, "k": n, "slices": s, "complex": True, "zmode": args.zmode,
                   "digits": digits,
                   "inputs": "seed 0, (N(0,1) + i N(0,1)) * 2^e_row, e_row ~ randint(-20, 20)"},
        "roofline": {"bound": "mfma", "achieved": round(achieved, 2), "peak": INT8_PEAK_TOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / INT8_PEAK_TOPS, 4), "traffic": traffic_for(workload),
                     "kernel": "gemm_kernel (INT8 ops of the s(s+1)/2 slice pairs)", "launches_per_step": launches,
                     "avg_ms": round(gemm_avg_ms, 4), "split_avg_ms": round(split_ms / calls, 4)},
    }

    if not args.no_native:
        tA = torch.from_numpy(A).cuda()
        tB = torch.from_numpy(B).cuda()
        for _ in range(3):
            tC = tA @ tB
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            tC = tA @ tB
        e1.record(stream)
        torch.cuda.synchronize()
        nms = e0.elapsed_time(e1) / args.steps
        Cn = tC.cpu().numpy()
        rel = float(np.linalg.norm(C_gpu - Cn) / np.linalg.norm(Cn))
        out["native_fp64"] = {"tflops": round(flops / (nms * 1e-3) / 1e12, 3), "ms": round(nms, 4),
                              "kind": "torch complex128 matmul (rocBLAS zgemm)"}
        out["rel_err_vs_native"] = rel
        out["meets_tolerance"] = bool(rel <= 1e-12)
        out["speedup_vs_native"] = round(nms / ms, 3)
    if args.copy_probe:
        x = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
        y = x.clone()
        torch.cuda.synchronize()
        del x, y
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(A, B, s, C_gpu, args.cpu_rows, args.zmode, args.digits == 1,
                                           C_native=None if args.no_native else Cn)
    oz.oz_destroy(h)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
