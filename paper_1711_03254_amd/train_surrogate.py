"""Trains the warm-start surrogate on near-steady states the solver
generates and compares cold and warm solves on held-out subvolumes at equal
accuracy.  Needs a GPU:

    python -m paper_1711_03254_amd.train_surrogate --out DIR

Writes DIR/surrogate.npz (FP32 weights, base width, levels, velocity and
density scales) and DIR/report.json (training loss per epoch, and per
held-out case and storage precision the steps and seconds of the cold and
the warm solve to each accuracy target against a long cold FP64 solve).
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np


def parse_targets(text):
    """'eu,ea;eu,ea' -> [(eu, ea), ...]"""
    return [tuple(float(v) for v in pair.split(",")) for pair in text.split(";")]


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--n-train", type=int, default=16)
    ap.add_argument("--size", type=int, default=128)
    ap.add_argument("--steps", type=int, default=60000, help="FP64 steps of a training sample")
    ap.add_argument("--n-eval", type=int, default=2)
    ap.add_argument("--ref-steps", type=int, default=200000, help="FP64 steps of the reference state")
    ap.add_argument("--max-steps", type=int, default=40000, help="step limit of a judged solve")
    ap.add_argument("--targets", default="0.04,0.004;0.02,0.001",
                    help="accuracy targets 'eps_u,eps_rhoA;...' against the reference")
    ap.add_argument("--epochs", type=int, default=150)
    ap.add_argument("--base", type=int, default=32)
    ap.add_argument("--lr", type=float, default=5e-4)
    ap.add_argument("--seed", type=int, default=100)
    ap.add_argument("--eval-seed", type=int, default=10100)
    ap.add_argument("--train-seconds", type=float, default=None, help="stop training after this long")
    args = ap.parse_args(argv)

    import torch  # noqa: F401
    from . import inputs, lbm, surrogate, warmstart as ws
    lbm.load_library()
    os.makedirs(args.out, exist_ok=True)
    phys = ws.physics()
    targets = parse_targets(args.targets)
    t0 = time.perf_counter()
    samples = []
    for k in range(args.n_train):
        s = ws.steady_sample(args.size, args.seed + k, phys, steps=args.steps)
        samples.append(s)
        print(f"# sample {k}: {s['info']} residual {s['residual']} ({time.perf_counter() - t0:.1f} s)", flush=True)
    t_data = time.perf_counter() - t0
    net = surrogate.Surrogate(base=args.base, seed=args.seed)
    net.u_scale = ws.u_scale_of(samples, phys)
    net.rho_scale = ws.rho_scale_of(samples)
    t0 = time.perf_counter()
    hist = ws.train(net, samples, phys, args.epochs, args.lr, time_budget=args.train_seconds,
                    log=lambda e, l: print(f"# epoch {e} loss {l:.5g} at {time.perf_counter() - t0:.1f} s", flush=True))
    t_train = time.perf_counter() - t0
    net.save(os.path.join(args.out, "surrogate.npz"))
    del samples
    evals = []
    for k in range(args.n_eval):
        seed = args.eval_seed + k
        solid, ra0, rb0, info = inputs.mixture_case(args.size, seed)
        t = time.perf_counter()
        ref_a, ref_u, ref_res = ws.reference(solid, ra0, rb0, phys, args.ref_steps)
        print(f"# eval {k}: reference {args.ref_steps} steps, residual {ref_res} "
              f"({time.perf_counter() - t:.1f} s)", flush=True)
        row = {"seed": seed, "info": info, "reference_residual": ref_res}
        row.update(ws.compare(net, dict(solid=solid, ra0=ra0, rb0=rb0), phys, (ref_a, ref_u), targets,
                              max_steps=args.max_steps))
        evals.append(row)
        print(f"# eval {k}: prediction {row['prediction_distance']} "
              + " ".join(f"{p}: {json.dumps(row[p]['factors'])}" for p in ("fp32", "fp16s")), flush=True)
    report = {
        "workload": {"physics": {k: list(v) if isinstance(v, tuple) else v for k, v in phys.items()},
                     "train": f"{args.n_train} mixture subvolumes {args.size}^3 (seeds {args.seed}..), radius (6, 16), "
                              f"porosity (0.3, 0.5), A fraction (0.1, 0.9); FP64 states after {args.steps} steps",
                     "eval": f"{args.n_eval} held-out subvolumes {args.size}^3 (seeds {args.eval_seed}..); reference: "
                             f"{args.ref_steps} cold FP64 steps; solves judged every 500 steps up to {args.max_steps}"},
        "network": {"base": args.base, "levels": surrogate.LEVELS, "params": net.n_params, "u_scale": net.u_scale,
                    "rho_scale": net.rho_scale},
        "training": {"epochs": len(hist), "lr": args.lr, "loss": hist, "data_seconds": t_data,
                     "train_seconds": t_train},
        "eval": evals,
    }
    with open(os.path.join(args.out, "report.json"), "w") as fh:
        json.dump(report, fh, indent=1)
    print("# done", flush=True)


if __name__ == "__main__":
    main()
