"""Autotuner of the batched GEMM plans (run on the GPU).

For every size bucket n and slice count s it builds a batch of square
complex problems of that size, and times its graph replay under each
candidate GEMM configuration: block shape (1 = 128 x 64 of 8 one-tile waves
with a 3-stage LDS ring, 2 = 64 x 64 with 2 stages, 4 = 128 x 64 of 4 waves
owning two 32-row tiles each -- s <= 6 only) and tile order (0 = by work,
problem by problem; 1 = whole problems dealt to per-XCD queues).  A candidate is forced
by loading a one-entry table before planning.  The fastest candidate of each
bucket goes into the table (JSON), together with every measured time.

    python -m paper_2503_22875_amd.autotune [--out PATH] [--sizes 32,64,...] [--slices 6,7]
"""
import argparse
import json
import os
import tempfile
import time

import numpy as np


def _rocm_version():
    try:
        return open("/opt/rocm/.info/version").read().strip()
    except OSError:
        return "unknown"


def _batch(n, count, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        A = np.asfortranarray(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
        B = np.asfortranarray(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
        out.append((A, B))
    return out


def time_config(oz, torch, handle, stream, dev, n, s, tile, order, reps):
    """Milliseconds per replay of one batch with a forced (tile, order)."""
    with tempfile.NamedTemporaryFile("w", suffix=".json", delete=False) as f:
        json.dump({"entries": [{"complex": 1, "n": n, "s": s, "tile": tile, "order": order}]}, f)
        path = f.name
    try:
        oz.oz_load_tuning(handle, path)
        cnt = len(dev)
        plan = oz.oz_gemm_batched_plan(handle, 1, "N" * cnt, "N" * cnt, [n] * cnt, [n] * cnt, [n] * cnt,
                                       [1.0] * cnt, [d[0] for d in dev], [n] * cnt, [d[1] for d in dev], [n] * cnt,
                                       [0.0] * cnt, [d[2] for d in dev], [n] * cnt, p=oz.prec(s))
        try:
            for _ in range(3):
                oz.oz_batch_graph_launch(plan)
            stream.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                oz.oz_batch_graph_launch(plan)
            e1.record(stream)
            stream.synchronize()
            return e0.elapsed_time(e1) / reps
        finally:
            oz.oz_batch_destroy(plan)
    finally:
        os.unlink(path)
        oz.oz_load_tuning(handle, "")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune", "gfx950.json"))
    ap.add_argument("--sizes", default="32,64,128,256,512")
    ap.add_argument("--slices", default="6,7")
    ap.add_argument("--reps", type=int, default=10)
    args = ap.parse_args()

    import torch

    import paper_2503_22875_amd as oz

    torch.cuda.set_device(0)
    props = torch.cuda.get_device_properties(0)
    stream = torch.cuda.Stream()
    handle = oz.oz_create(0)
    oz.oz_set_stream(handle, stream.cuda_stream)
    entries = []
    t_start = time.time()
    for n in [int(x) for x in args.sizes.split(",")]:
        count = int(max(8, min(512, (1 << 28) // (n ** 3))))
        probs = _batch(n, count, seed=n)
        dev = [(torch.from_numpy(A.ravel(order="F")).cuda(), torch.from_numpy(B.ravel(order="F")).cuda(),
                torch.zeros(n * n, dtype=torch.complex128, device="cuda")) for A, B in probs]
        torch.cuda.synchronize()
        for s in [int(x) for x in args.slices.split(",")]:
            timings = {}
            for tile in ((1, 2, 4) if s <= 6 else (1, 2)):
                for order in (0, 1):
                    timings["tile%d_order%d" % (tile, order)] = time_config(oz, torch, handle, stream, dev, n, s,
                                                                            tile, order, args.reps)
            best = min(timings, key=timings.get)
            flops = 8.0 * n ** 3 * count
            ent = {"complex": 1, "n": n, "s": s, "tile": int(best[4]), "order": int(best[-1]), "count": count,
                   "tflops": round(flops / (timings[best] * 1e-3) / 1e12, 2)}
            ent.update({"ms_" + key: round(val, 4) for key, val in sorted(timings.items())})
            entries.append(ent)
            print("n=%4d s=%d count=%3d best %s %.3f ms  (%s)" % (
                n, s, count, best, timings[best], ", ".join("%s %.3f" % kv for kv in sorted(timings.items()))),
                flush=True)
        del dev
    oz.oz_destroy(handle)
    out = {"device": props.gcnArchName.split(":")[0], "cus": props.multi_processor_count, "rocm": _rocm_version(),
           "torch": torch.__version__, "generated_by": "python -m paper_2503_22875_amd.autotune",
           "seconds": round(time.time() - t_start, 1), "entries": entries}
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    with open(args.out, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", args.out)


if __name__ == "__main__":
    main()
