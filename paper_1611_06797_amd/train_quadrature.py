"""Train the learned Laplace-quadrature network on the GPU.

Dataset: seeded (splitmix64) samples, x_min log-uniform in [0.05, 1] Ha,
x_max / x_min log-uniform in [10, 1e4], n_tau in {6, 8, 10, 12}; targets
are the plain minimax fits (one continuation sweep per n_tau).  Training uses
the library's own forward / backward / Adam kernels.  Writes the weight file
and a JSON report (loss history, validation error, certification rate of the
polished proposals, timing of learned vs plain quadrature).

  python -m paper_1611_06797_amd.train_quadrature [--count 100000] [--epochs 200]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_OUT = os.path.join(HERE, "data", "laplace_mlp.bin")


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--count", type=int, default=100000)
    ap.add_argument("--val", type=int, default=2000)
    ap.add_argument("--epochs", type=int, default=200)
    ap.add_argument("--batch", type=int, default=1024)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default=DEFAULT_OUT)
    args = ap.parse_args(argv)

    sys.path.insert(0, os.path.dirname(HERE))
    from paper_1611_06797_amd import ltmp2 as L

    t0 = time.time()
    X, Y, M, xr = L.mlp_dataset(args.count, args.seed)
    t_data = time.time() - t0
    print(f"[train] dataset {args.count} in {t_data:.1f}s", flush=True)
    Xv, Yv, Mv, xrv = L.mlp_dataset(args.val, args.seed + 1)
    params = L.mlp_init(args.seed)
    t0 = time.time()
    hist = L.mlp_train(params, X, Y, M, args.epochs, args.batch, args.lr, args.seed)
    t_train = time.time() - t0
    print(f"[train] {args.epochs} epochs in {t_train:.1f}s: loss {hist[0]:.3e} -> {hist[-1]:.3e}",
          flush=True)
    out = L.mlp_forward(params, Xv)
    err = np.abs(out - Yv)[Mv > 0]
    val_mse = float((err ** 2).mean())
    print(f"[train] validation mse {val_mse:.3e}, max |err| {err.max():.3e}", flush=True)

    # certification of the polished proposals and timing against the plain fit
    ncheck = min(200, args.val)
    cert = 0
    t_learn = 0.0
    t_plain = 0.0
    rel_gap = []
    for k in range(ncheck):
        n = int(round(Xv[k, 2] * 12))
        a, b = xrv[k]
        t1 = time.perf_counter()
        tau, w, d, fl = L.learned_quadrature(params, a, b, n)
        t2 = time.perf_counter()
        tp, wp, dp = L.quadrature(a, b, n)
        t3 = time.perf_counter()
        cert += fl & 1
        t_learn += t2 - t1
        t_plain += t3 - t2
        rel_gap.append(abs(d - dp) / dp)
    report = {
        "count": args.count, "epochs": args.epochs, "batch": args.batch, "lr": args.lr,
        "seed": args.seed, "dataset_seconds": t_data, "train_seconds": t_train,
        "loss_first": float(hist[0]), "loss_last": float(hist[-1]),
        "loss_history": [float(v) for v in hist],
        "validation_mse": val_mse, "validation_max_abs_err": float(err.max()),
        "certified_fraction": cert / ncheck, "checked": ncheck,
        "mean_learned_ms": 1e3 * t_learn / ncheck, "mean_plain_ms": 1e3 * t_plain / ncheck,
        "max_rel_delta_gap": float(max(rel_gap)),
    }
    print(f"[train] certified {cert}/{ncheck}; learned {report['mean_learned_ms']:.2f} ms vs "
          f"plain {report['mean_plain_ms']:.2f} ms per fit", flush=True)
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    L.write_mlp_weights(args.out, params)
    with open(os.path.splitext(args.out)[0] + ".json", "w") as f:
        json.dump(report, f, indent=1)
    print(json.dumps({k: v for k, v in report.items() if k != "loss_history"}), flush=True)


if __name__ == "__main__":
    main()
