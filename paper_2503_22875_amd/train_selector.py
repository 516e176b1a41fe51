"""Train the learned slice-count selector on the GPU (run from the repository root).

    python -m paper_2503_22875_amd.train_selector [--count 50000] [--holdout 5000] [--epochs 80]

1. Draws the instance table (m, n, k log-uniform in [64, 2048] rounded to 16;
   exponent spread 0..40 per entry / per vector / half and half; full or
   shortened significands; optional zeros; two value families; four
   tolerances log-uniform in [1e-15, 1e-4] per instance) with
   ``workloads.selector_instances``.
2. Generates and labels every instance on the GPU (``oz_selector_dataset``):
   the library draws the operands, runs the s_ref = 12 emulation once keeping
   its INT32 anti-diagonal sums, forms every C_s from them, and labels each
   tolerance with the smallest s whose scale-weighted error against C_12 meets it.
3. Trains the 16-64-64-1 network on the GPU (``oz_mlp_train``, pinball loss
   tau = 0.9, Adam) on the training rows, evaluates on the held-out rows
   against the labels and against the statistics rule, and writes the network
   (``tune/selector_gfx950.bin``) and a JSON report beside it.
"""
import argparse
import json
import math
import os
import time

import numpy as np


def pairs(s):
    return s * (s + 1) // 2


def start_cost(start, label):
    """(slice pairs computed, check rounds) of a tolerance-driven call that
    starts at `start` and ends at max(start, label)."""
    final = np.maximum(start, label)
    return pairs(final), 1 + np.maximum(0, label - start)


def evaluate(pred, label, name):
    pred = np.asarray(pred, np.int64)
    label = np.asarray(label, np.int64)
    pw, rounds = start_cost(pred, label)
    return {
        "selector": name,
        "exact": float(np.mean(pred == label)),
        "under": float(np.mean(pred < label)),
        "over": float(np.mean(pred > label)),
        "mean_abs_diff": float(np.mean(np.abs(pred - label))),
        "mean_pairs": float(np.mean(pw)),
        "mean_check_rounds": float(np.mean(rounds)),
        "pairs_vs_oracle_choice": float(np.sum(pw) / np.sum(pairs(label))),
    }


def main():
    ap = argparse.ArgumentParser()
    here = os.path.dirname(os.path.abspath(__file__))
    ap.add_argument("--count", type=int, default=50000)
    ap.add_argument("--holdout", type=int, default=5000)
    ap.add_argument("--chunk", type=int, default=2500)
    ap.add_argument("--s-ref", type=int, default=12)
    ap.add_argument("--epochs", type=int, default=80)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--tau", type=float, default=0.9)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=2503)
    ap.add_argument("--out", default=os.path.join(here, "tune", "selector_gfx950.bin"))
    args = ap.parse_args()

    import torch

    import paper_2503_22875_amd as oz
    import workloads

    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    h = oz.oz_create(0)
    oz.oz_set_stream(h, stream.cuda_stream)
    total = args.count + args.holdout
    params, tols = workloads.selector_instances(total, seed=args.seed)
    ntol = tols.shape[1]
    rows = total * ntol
    X = torch.empty(rows * 16, dtype=torch.float32, device="cuda")
    y = torch.empty(rows, dtype=torch.float32, device="cuda")
    s_rule = np.empty(rows, np.int64)
    eps = np.empty((total, args.s_ref))
    t0 = time.time()
    for c0 in range(0, total, args.chunk):
        c1 = min(total, c0 + args.chunk)
        sr, ep = oz.oz_selector_dataset(h, params[c0:c1], tols[c0:c1], X[c0 * ntol * 16:],
                                        y[c0 * ntol:], s_ref=args.s_ref)
        s_rule[c0 * ntol:c1 * ntol] = sr
        eps[c0:c1] = np.asarray(ep)
        print("labelled %d / %d instances, %.1f s" % (c1, total, time.time() - t0), flush=True)
    t_label = time.time() - t0
    n_train = args.count * ntol
    labels = y.cpu().numpy().astype(np.int64)

    net = oz.oz_mlp_create(h, args.seed)
    oz.oz_mlp_fit_norm(net, n_train, X)
    t0 = time.time()
    losses = []
    # two phases: the learning rate drops by 5x for the last quarter of the epochs
    e1 = (3 * args.epochs) // 4
    for ep_count, lr in ((e1, args.lr), (args.epochs - e1, args.lr / 5)):
        if ep_count:
            losses += oz.oz_mlp_train(net, n_train, X, y, ep_count, args.batch, args.tau, lr,
                                      args.seed + len(losses))
        print("epochs %d, loss %.4f, %.1f s" % (len(losses), losses[-1], time.time() - t0), flush=True)
    t_train = time.time() - t0

    # held-out evaluation
    yp = torch.empty(rows - n_train, dtype=torch.float32, device="cuda")
    oz.oz_mlp_forward(net, rows - n_train, X[n_train * 16:], yp)
    torch.cuda.synchronize()
    pred = np.clip(np.floor(yp.cpu().numpy() + 0.5), 2, args.s_ref).astype(np.int64)
    lab = labels[n_train:]
    rule = np.maximum(s_rule[n_train:], 2)
    report = {
        "device": torch.cuda.get_device_properties(0).gcnArchName.split(":")[0],
        "instances": {"train": args.count, "holdout": args.holdout, "tolerances_each": ntol, "seed": args.seed},
        "s_ref": args.s_ref, "epochs": args.epochs, "batch": args.batch, "tau": args.tau, "lr": args.lr,
        "label_seconds": round(t_label, 1), "train_seconds": round(t_train, 1),
        "loss_first": losses[0], "loss_last": losses[-1],
        "label_histogram": np.bincount(labels, minlength=args.s_ref + 1).tolist(),
        "holdout": [evaluate(pred, lab, "learned"), evaluate(rule, lab, "rule"),
                    evaluate(np.full_like(lab, 2), lab, "escalate_from_2"),
                    evaluate(np.full_like(lab, int(lab.max())), lab, "fixed_max")],
    }
    for r in report["holdout"]:
        print(json.dumps(r), flush=True)
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    oz.oz_mlp_save(net, args.out)
    with open(os.path.splitext(args.out)[0] + ".json", "w") as f:
        json.dump(report, f, indent=1)
    print("wrote", args.out, flush=True)
    oz.oz_mlp_destroy(net)
    oz.oz_destroy(h)
    if not math.isfinite(losses[-1]):
        raise SystemExit("training diverged")


if __name__ == "__main__":
    main()
