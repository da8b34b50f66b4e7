"""Trains the warm-start surrogate on steady states the solver generates and
compares cold and warm solves on held-out subvolumes.  Needs a GPU:

    python -m paper_1711_03254_amd.train_surrogate --out DIR

Writes DIR/surrogate.npz (FP32 weights, base width, velocity scale) and
DIR/report.json (training loss per epoch, and per held-out sample the steps
and seconds to the residual for the cold and the warm start, the prediction
errors and the difference of the two converged states).
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--n-train", type=int, default=24)
    ap.add_argument("--train-size", type=int, default=64)
    ap.add_argument("--n-eval", type=int, default=3)
    ap.add_argument("--eval-size", type=int, default=128)
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--base", type=int, default=32)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed", type=int, default=100)
    ap.add_argument("--tol64", type=float, default=1e-6)
    ap.add_argument("--tol32", type=float, default=1e-5)
    ap.add_argument("--train-seconds", type=float, default=None, help="stop training after this long")
    args = ap.parse_args(argv)

    import torch  # noqa: F401
    from . import lbm, surrogate, warmstart as ws
    lbm.load_library()
    os.makedirs(args.out, exist_ok=True)
    phys = ws.physics()
    scale = args.train_size / 128.0
    rr_train = (6.0 * scale, 16.0 * scale)
    t0 = time.perf_counter()
    samples = []
    for k in range(args.n_train):
        s = ws.steady_sample(args.train_size, args.seed + k, phys, tol=1e-7, prec="fp64", max_steps=30000,
                             radius_range=rr_train)
        samples.append(s)
        print(f"# sample {k}: {s['info']} steps {s['steps']} converged {s['converged']} "
              f"({time.perf_counter() - t0:.1f} s)", flush=True)
    t_data = time.perf_counter() - t0
    net = surrogate.Surrogate(base=args.base, seed=args.seed)
    net.u_scale = ws.u_scale_of(samples, phys)
    t0 = time.perf_counter()
    hist = ws.train(net, samples, phys, args.epochs, args.lr, time_budget=args.train_seconds,
                    log=lambda e, l: print(f"# epoch {e} loss {l:.5g} at {time.perf_counter() - t0:.1f} s", flush=True))
    t_train = time.perf_counter() - t0
    net.save(os.path.join(args.out, "surrogate.npz"))

    evals = []
    for k in range(args.n_eval):
        seed = args.seed + 10000 + k
        solid, ra0, rb0, info = ws.inputs.mixture_case(args.eval_size, seed)
        sample = dict(solid=solid, ra0=ra0, rb0=rb0)
        row = {"seed": seed, "info": info}
        row["fp64"] = ws.compare(net, sample, phys, args.tol64, prec="fp64")
        row["fp32"] = ws.compare(net, sample, phys, args.tol32, prec="fp32")
        evals.append(row)
        print(f"# eval {k}: {json.dumps(row)}", flush=True)
    report = {
        "workload": {"physics": {k: list(v) if isinstance(v, tuple) else v for k, v in phys.items()},
                     "train": f"{args.n_train} mixture subvolumes {args.train_size}^3, radius {rr_train}, "
                              f"porosity (0.3, 0.5), A fraction (0.1, 0.9); FP64 steady states (residual 1e-7, at most 30000 steps)",
                     "eval": f"{args.n_eval} held-out subvolumes {args.eval_size}^3, radius (6, 16)"},
        "network": {"base": args.base, "params": net.n_params, "u_scale": net.u_scale},
        "training": {"epochs": args.epochs, "lr": args.lr, "loss": hist, "data_seconds": t_data,
                     "train_seconds": t_train},
        "tolerances": {"fp64": args.tol64, "fp32": args.tol32},
        "eval": evals,
    }
    for prec in ("fp64", "fp32"):
        c = np.mean([e[prec]["cold_steps"] for e in evals])
        w = np.mean([e[prec]["warm_steps"] for e in evals])
        report[f"mean_steps_{prec}"] = {"cold": c, "warm": w, "factor": c / w}
    with open(os.path.join(args.out, "report.json"), "w") as fh:
        json.dump(report, fh, indent=1)
    print(json.dumps({k: v for k, v in report.items() if k.startswith("mean_steps")}), flush=True)


if __name__ == "__main__":
    main()
