"""Throughput of the fused two-component Shan-Chen D3Q19 step on one MI355X.

Workload: the 1 % mixture in packed spheres -- a 256^3 periodic lattice
filled with seeded non-overlapping spheres of radius 12 at porosity 0.40
(solid mask), droplets of component A (radius 4, 1 % of the pore volume) in
a carrier B with droplet interfaces of tanh width 1.5; nu_B = 1/6,
nu_A = 1/60 (ratio 10); G = -4.2; body force 1e-6 along z; wall parameter
rho^s = 0.25.  A step is one launch of the fused
kernel over the whole lattice (pull-stream with bounce-back, moments, LDS
pseudo-potential halo, Shan-Chen force, regularized collision with the
forcing term), with the FP64 mass / finiteness check every 100 steps.

MLUPS counts fluid-site updates (solid sites hold no populations and are
skipped).  Algorithmic bytes per update: 2 components x 19 populations x
(read + write) x storage size = 304 B at FP32.  The printed JSON line gives
FP32 as `value`; FP64, FP16-shifted and BF16-shifted storage are measured
the same way under `precisions`.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "MLUPS and % HBM peak (FP32 vs FP16-shifted); time-to-steady-state w/ warm start"
KERNEL_SRC = os.path.join(ROOT, "paper_1711_03254_amd", "csrc", "lbm_kernels.hip")
LAYOUT_SRC = os.path.join(ROOT, "paper_1711_03254_amd", "csrc", "lbm_api.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_step_fp32_packed_spheres_256.json")


def workload(n=256, G=-4.2, width=1.5):
    from paper_1711_03254_amd import inputs
    solid, rA, rB, info = inputs.packed_spheres_case(n=n, radius=12.0, porosity=0.40, drop_radius=4.0,
                                                     drop_fraction=0.01, seed=3, minority=0.03,
                                                     interface_width=width)
    rA[solid == 1] = 0.0
    rB[solid == 1] = 0.0
    phys = dict(tau=(1.0 / 60.0 / (1.0 / 3.0) + 0.5, 1.0), G=G, g=(0.0, 0.0, 1e-6), rho_s=0.25)
    return solid, rA, rB, info, phys


def kernel_hash():
    """Digest of the step kernel and of the host code that lays out its data
    (both decide the traffic the counters saw), over their code lines only."""
    from paper_1711_03254_amd.build import source_digest
    return source_digest()


def time_precision(lbm, torch, prec, solid, rA, rB, phys, steps, warmup, check_every):
    # The library launches on the stream it is given; events are recorded on
    # that same stream so that they bracket its kernels.
    stream = torch.cuda.Stream()
    n = solid.shape[0]
    ctx = lbm.lbm_init(lbm.Params(n, n, n, prec=lbm.PRECISIONS[prec], solid=solid, rho_init=(rA, rB),
                                  check_every=check_every, stream=stream, **phys))
    info = lbm.lbm_info(ctx)
    lbm.lbm_step(ctx, warmup)
    torch.cuda.synchronize()
    # (1) the whole step as a user runs it, periodic checks included
    t0 = time.perf_counter()
    lbm.lbm_step(ctx, steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # (2) the step kernel alone: HIP events on the stream the kernel runs on
    ctx2 = lbm.lbm_init(lbm.Params(n, n, n, prec=lbm.PRECISIONS[prec], solid=solid, rho_init=(rA, rB),
                                   check_every=0, stream=stream, **phys))
    lbm.lbm_step(ctx2, warmup)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    lbm.lbm_step(ctx2, steps)
    e1.record(stream)
    torch.cuda.synchronize()
    kern_ms = e0.elapsed_time(e1) / steps
    red = lbm.lbm_reduce(ctx)
    drift = [abs(red[k] - info["mass0"][k]) / info["mass0"][k] for k in range(2)]
    lbm.lbm_free(ctx)
    lbm.lbm_free(ctx2)
    nf = info["n_fluid"]
    bpl = info["bytes_per_lu"]
    ms_step = wall / steps * 1e3
    return {
        "mlups": nf / (ms_step * 1e-3) / 1e6,
        "ms_per_step": ms_step,
        "kernel_ms": kern_ms,
        "kernel_mlups": nf / (kern_ms * 1e-3) / 1e6,
        "bytes_per_lu": bpl,
        "algorithmic_GBs": nf * bpl / (kern_ms * 1e-3) / 1e9,
        "hbm_frac": nf * bpl / (kern_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "mass_drift": max(drift),
        "n_fluid": nf,
        "tile": list(info["tile"]),
        "zchunk": info["zchunk"],
        "blocks": info["blocks"],
    }


def cpu_baseline(solid, rA, rB, phys, steps=3):
    """The FP64 oracle on the same lattice, timed on the host: on the threads
    the job is given (OMP_NUM_THREADS; the box allots 16 host threads per GPU)
    for `steps` steps, and on one thread for one step."""
    from oracle import oracle as ora
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count() or 1
    n = solid.shape[0]
    p = ora.Params(n, n, n, solid=solid, **phys)
    f = ora.init(p, rA, rB)
    nf = int((solid == 0).sum())
    out = {}
    for nthr, k in ((threads, steps), (1, 1)):
        ora.set_threads(nthr)
        t0 = time.perf_counter()
        ora.run(p, f, k)
        dt = time.perf_counter() - t0
        out[nthr] = (nf * k / dt / 1e6, ora.get_threads(), k, dt)
    ora.set_threads(threads)
    v, used, k, dt = out[threads]
    v1, _, k1, dt1 = out[1]
    return {"value": v, "unit": "MLUPS", "cores": used, "kind": "oracle",
            "sample": f"the full {n}^3 workload, {k} steps of the FP64 oracle on {used} threads ({dt:.1f} s)",
            "one_thread": {"value": v1, "unit": "MLUPS", "cores": 1,
                           "sample": f"the full {n}^3 workload, {k1} step on one thread ({dt1:.1f} s)"},
            "host_cpus": os.cpu_count()}


TUNED = os.path.join(ROOT, "paper_1711_03254_amd", "tuned", "launch_shapes.json")


def ensemble(lbm, torch, steps, warmup, tune=False):
    """The batched ensemble: 64 ducts of uneven sizes stepped by one
    graph-replayed launch per step, against the same domains stepped one
    launch each.  FP32; MLUPS over all fluid sites; wall clock with the
    device synchronized on both sides (the batch runs on its own stream).
    The launch shape is the autotuner's, from its committed cache (tune=True
    tunes first and rewrites the cache)."""
    from paper_1711_03254_amd import autotune, inputs
    doms = inputs.ensemble_case(64)
    if tune:
        autotune.tune_batch(doms, "fp32", cache=TUNED)
    shape = autotune.cached_batch_shape(doms, "fp32", TUNED)
    tile, zc = (tuple(shape["tile"]), shape["zchunk"]) if shape else ((64, 8), 0)
    stream = torch.cuda.Stream()
    ctxs = []
    for d in doms:
        nz, ny, nx = d["shape"]
        ctxs.append(lbm.lbm_init(lbm.Params(nx, ny, nz, prec=lbm.LBM_FP32, solid=d["solid"],
                                            rho_init=(d["rho_A"], d["rho_B"]), tau=d["tau"], G=d["G"], g=d["g"],
                                            rho_s=d["rho_s"], stream=stream, tile=tile, zchunk=zc)))
    nf = sum(lbm.lbm_info(c)["n_fluid"] for c in ctxs)
    for c in ctxs:
        lbm.lbm_step(c, warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for c in ctxs:
        lbm.lbm_step(c, steps)
    torch.cuda.synchronize()
    t_single = time.perf_counter() - t0
    b = lbm.lbm_batch_create(ctxs)
    lbm.lbm_batch_step(b, warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lbm.lbm_batch_step(b, steps)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    lbm.lbm_batch_free(b)
    for c in ctxs:
        lbm.lbm_free(c)
    out = {"domains": len(doms), "n_fluid": nf, "steps": steps,
           "launch": {"tile": list(tile), "zchunk": zc, "tuned": shape is not None}}
    for name, t in (("batched", t_batch), ("one_launch_per_domain", t_single)):
        mlups = nf * steps / t / 1e6
        out[name] = {"ms_per_step": round(t / steps * 1e3, 4), "mlups": round(mlups, 1),
                     "hbm_frac": round(mlups * 1e6 * 304 / 1e9 / HBM_PEAK_GBS, 4)}
    return out


WEIGHTS = os.path.join(ROOT, "paper_1711_03254_amd", "weights", "surrogate_coupled_128.npz")
WARM_TARGETS = ((0.04, 0.004), (0.02, 0.001))


def warm_start(lbm):
    """Time to steady state at equal accuracy, cold and with the learned warm
    start, on one held-out 128^3 mixture subvolume with the coupling on
    (the surrogate's workload), FP32 and FP16S storage: steps and seconds
    to each accuracy target (eps_u, eps_rhoA) against the state of 200 000
    cold FP64 steps, for the cold start, the consistent restart of the cold
    fields (u_F = 0), the network's velocity alone and the network's
    velocity and densities."""
    from paper_1711_03254_amd import inputs, surrogate, warmstart as ws
    if not os.path.exists(WEIGHTS):
        return None
    net = surrogate.Surrogate.load(WEIGHTS)
    phys = ws.physics()
    solid, ra0, rb0, info = inputs.mixture_case(128, 10100)
    ref_a, ref_u, ref_res = ws.reference(solid, ra0, rb0, phys, 200000)
    r = ws.compare(net, dict(solid=solid, ra0=ra0, rb0=rb0), phys, (ref_a, ref_u), WARM_TARGETS)
    out = {"workload": f"mixture subvolume 128^3, seed 10100, {json.dumps(info)}, G={phys['G']}, g={phys['g'][2]} z, "
                       f"reference: 200000 cold FP64 steps (last-100-step residual {ref_res[0]:.2e} in u_F)",
           "network": {"params": net.n_params, "weights": os.path.relpath(WEIGHTS, ROOT)},
           "targets": [list(t) for t in WARM_TARGETS], "predict_seconds": round(r["predict_seconds"], 4),
           "prediction_distance": r["prediction_distance"]}
    for prec in ("fp32", "fp16s"):
        row = {}
        for arm in ("cold", "cold_consistent", "warm_u", "warm"):
            a = r[prec][arm]
            row[arm] = {"reached": a["reached"], "final": [round(v, 6) for v in a["final"]]}
        row["factors"] = r[prec]["factors"]
        out[prec] = row
    return out


def traffic_for(kernel, n_fluid):
    """HBM bytes per step launch from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source, the same kernel
    instance and the same workload; else None."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    t = json.load(open(TRAFFIC_FILE))
    if t.get("kernel_and_layout_source_sha256_16") != kernel_hash() or t.get("kernel") != kernel:
        return None
    if f"{n_fluid} fluid sites" not in t.get("workload", ""):
        return None
    return t.get("hbm_bytes_per_launch")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--precisions", default="fp32,fp16s,bf16s,fp64")
    ap.add_argument("--check-every", type=int, default=100)
    ap.add_argument("--size", type=int, default=256)
    ap.add_argument("--G", type=float, default=-4.2)
    ap.add_argument("--interface-width", type=float, default=1.5)
    ap.add_argument("--no-ensemble", dest="ensemble", action="store_false",
                    help="skip the batched 64-domain ensemble")
    ap.add_argument("--no-warm-start", dest="warm_start", action="store_false",
                    help="skip the cold / warm time-to-steady-state comparison")
    ap.add_argument("--no-all-fluid", dest="all_fluid", action="store_false",
                    help="skip the all-fluid lattice of the same size")
    ap.add_argument("--tune", action="store_true",
                    help="autotune the ensemble's launch shape and rewrite the committed cache")
    ap.add_argument("--copy-probe-gib", type=float, default=0.0,
                    help="also run a plain device copy of this many GiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures the step on one MI355X; runs on several GPUs are not supported "
              f"(asked for {args.gpus}).", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1711_03254_amd.lbm as lbm
    lbm.load_library()
    torch.cuda.set_device(0)

    if args.copy_probe_gib > 0:
        nel = int(args.copy_probe_gib * 2 ** 30 / 4)
        src = torch.ones(nel, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):   # an elementwise kernel: reads nel * 4 bytes, writes nel * 4 bytes
            torch.mul(src, 2.0, out=dst)
        torch.cuda.synchronize()
        print(f"# copy probe: 3 elementwise copies of {nel * 4} bytes", file=sys.stderr, flush=True)
        del src, dst

    solid, rA, rB, info, phys = workload(args.size, args.G, args.interface_width)
    print(f"# workload ready: {info}", file=sys.stderr, flush=True)
    res = {}
    for prec in args.precisions.split(","):
        k = args.steps if prec == "fp32" else max(50, args.steps // 2)
        res[prec] = time_precision(lbm, torch, prec, solid, rA, rB, phys, k, args.warmup, args.check_every)
        print(f"# {prec}: {json.dumps(res[prec])}", file=sys.stderr, flush=True)
    # The same kernel on an all-fluid lattice of the same size (a droplet of
    # A in B, no solids): its bandwidth fraction without the geometry's
    # partly solid tiles, whose lanes and ring pulls it spends on fewer sites.
    allf = {}
    if args.all_fluid:
        import numpy as np
        from paper_1711_03254_amd import inputs
        n = args.size
        dA, dB = inputs.droplet((n, n, n), n / 6.4)
        zero = np.zeros((n, n, n), np.uint8)
        phys_af = dict(tau=(1.0, 1.0), G=-3.0, g=(0.0, 0.0, 0.0), rho_s=0.0)
        for prec in ("fp32", "fp16s"):
            r = time_precision(lbm, torch, prec, zero, dA, dB, phys_af, max(50, args.steps // 2), args.warmup, 0)
            allf[prec] = {k: r[k] for k in ("kernel_ms", "kernel_mlups", "algorithmic_GBs", "hbm_frac")}
            print(f"# all-fluid {prec}: {json.dumps(allf[prec])}", file=sys.stderr, flush=True)
    ens = None
    if args.ensemble:
        ens = ensemble(lbm, torch, max(20, args.steps // 5), 4, tune=args.tune)
        print(f"# ensemble: {json.dumps(ens)}", file=sys.stderr, flush=True)
    ws_res = None
    if args.warm_start:
        ws_res = warm_start(lbm)
        print(f"# warm start: {json.dumps(ws_res)}", file=sys.stderr, flush=True)
    main_r = res["fp32"]
    n_fluid = main_r["n_fluid"]
    kname = "step_kernel<float,{},{},MODE_STEP>".format(*main_r["tile"])
    roof = {
        "bound": "hbm",
        "achieved": round(main_r["algorithmic_GBs"], 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(main_r["algorithmic_GBs"] / HBM_PEAK_GBS, 4),
        "traffic": traffic_for(kname, n_fluid),
        "kernel": kname,
        "algorithmic_bytes_per_launch": n_fluid * main_r["bytes_per_lu"],
        "kernel_ms": round(main_r["kernel_ms"], 4),
    }
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(solid, rA, rB, phys)
        print(f"# cpu baseline: {cpu}", file=sys.stderr, flush=True)
    line = {
        "metric": METRIC,
        "value": round(main_r["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_r["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"1% mixture in packed spheres, {args.size}^3 periodic, sphere radius 12, porosity "
                        f"{info['porosity']:.3f}, {info['droplets']} droplets of A (radius 4, tanh interface "
                        f"width {args.interface_width}), nu ratio 10, G={args.G}, g=1e-6 z, rho_s=0.25, "
                        f"FP32 storage, FP64 check every {args.check_every} steps",
            "n_fluid": n_fluid,
            "parallelism": "single GPU",
        },
        "hbm_frac": round(main_r["hbm_frac"], 4),
        "roofline": roof,
        "cpu_baseline": cpu,
        "all_fluid": {k: {kk: round(v, 4) for kk, v in r.items()} for k, r in allf.items()},
        "warm_start": ws_res,
        "ensemble": ens,
        "precisions": {k: {kk: (round(v, 4) if isinstance(v, float) else v) for kk, v in r.items()}
                       for k, r in res.items()},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
