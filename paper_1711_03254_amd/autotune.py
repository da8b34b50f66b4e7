"""Launch-shape autotuner for the fused step.

For a precision and a set of domains it times every compiled tile shape and a
few z-chunk depths through the C ABI (HIP events on a dedicated stream, after
warm-up steps) and keeps the fastest; results are cached in a JSON file keyed
by precision and domain shape, so a run pays for tuning once.

A batch shares one tile shape (one kernel instance per launch) but each domain
keeps its own z-chunk, so `tune_batch` picks the tile that minimizes the
summed step time of the domains, each at its best z-chunk.
"""
from __future__ import annotations

import json
import os

import numpy as np

TILES = ((64, 4), (64, 8), (64, 16), (32, 8), (32, 16), (16, 16), (8, 32))
ZCHUNKS = (8, 16, 32, 64)


def _key(prec: str, shape, fluid_fraction: float) -> str:
    nz, ny, nx = shape
    return f"{prec}:{nx}x{ny}x{nz}:fluid{round(fluid_fraction, 1)}"


def _time_config(lbm, torch, prec, dom, tile, zchunk, steps, warmup, stream):
    nz, ny, nx = dom["shape"]
    if tile[0] > 2 * nx and tile != TILES[-1]:
        return None  # a tile much wider than the lattice only idles lanes
    try:
        ctx = lbm.lbm_init(lbm.Params(nx, ny, nz, prec=lbm.PRECISIONS[prec], solid=dom["solid"],
                                      rho_init=(dom["rho_A"], dom["rho_B"]), tau=dom["tau"], G=dom["G"],
                                      g=dom["g"], rho_s=dom["rho_s"], stream=stream, tile=tile, zchunk=zchunk))
    except lbm.LBMError as e:
        if e.code == lbm.LBM_EINVAL:
            return None  # a tile this precision is not compiled for
        raise
    lbm.lbm_step(ctx, warmup)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    lbm.lbm_step(ctx, steps)
    e1.record(stream)
    torch.cuda.synchronize()
    lbm.lbm_free(ctx)
    return e0.elapsed_time(e1) / steps


def tune_domain(dom: dict, prec: str = "fp32", steps: int = 20, warmup: int = 4, cache: str | None = None,
                tiles=TILES, zchunks=ZCHUNKS) -> dict:
    """Best (tile, zchunk) for one domain; dom has shape, solid, rho_A, rho_B,
    tau, G, g, rho_s (as produced by paper_1711_03254_amd.inputs)."""
    import torch
    from . import lbm
    lbm.load_library()
    frac = float((np.asarray(dom["solid"]) == 0).mean()) if dom.get("solid") is not None else 1.0
    key = _key(prec, dom["shape"], frac)
    table = _load(cache)
    if key in table:
        return table[key]
    stream = torch.cuda.Stream()
    times = {}
    for tile in tiles:
        for zc in zchunks:
            if zc > dom["shape"][0]:
                continue
            t = _time_config(lbm, torch, prec, dom, tile, zc, steps, warmup, stream)
            if t is not None:
                times[f"{tile[0]}x{tile[1]}/{zc}"] = t
    best = min(times, key=times.get)
    tile, zc = best.split("/")
    res = {"tile": [int(v) for v in tile.split("x")], "zchunk": int(zc), "ms": times[best], "all": times}
    table[key] = res
    _save(cache, table)
    return res


def tune_batch(domains: list, prec: str = "fp32", steps: int = 10, warmup: int = 2, cache: str | None = None,
               tiles=TILES, zchunks=ZCHUNKS) -> dict:
    """One tile for the whole batch (the one minimizing the summed step time
    of the distinct domain shapes) and a z-chunk per domain."""
    per_shape = {}
    for d in domains:
        k = tuple(d["shape"])
        if k not in per_shape:
            per_shape[k] = (d, tune_domain(d, prec, steps, warmup, cache, tiles, zchunks))
    best_tile, best_total = None, None
    for tile in tiles:
        tname = f"{tile[0]}x{tile[1]}"
        total = 0.0
        for d in domains:
            allt = per_shape[tuple(d["shape"])][1]["all"]
            cand = [v for k, v in allt.items() if k.startswith(tname + "/")]
            if not cand:
                total = None
                break
            total += min(cand)
        if total is not None and (best_total is None or total < best_total):
            best_tile, best_total = tile, total
    zc = []
    for d in domains:
        allt = per_shape[tuple(d["shape"])][1]["all"]
        tname = f"{best_tile[0]}x{best_tile[1]}/"
        zc.append(int(min((k for k in allt if k.startswith(tname)), key=allt.get).split("/")[1]))
    return {"tile": list(best_tile), "zchunk": zc, "sum_ms": best_total}


def _load(path):
    if path and os.path.exists(path):
        with open(path) as fh:
            return json.load(fh)
    return {}


def _save(path, table):
    if path:
        tmp = path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(table, fh, indent=1, sort_keys=True)
        os.replace(tmp, path)
