"""Launch-shape autotuner for the fused step.

For a precision and a set of domains it times every compiled tile shape and a
few z-chunk depths through the C ABI (HIP events on a dedicated stream, after
warm-up steps) and keeps the fastest; results are cached in a JSON file keyed
by precision and domain shape, so a run pays for tuning once.

A batch shares one tile shape (one kernel instance per launch); `tune_batch`
times the whole batch at each candidate tile and z-chunk and keeps the
fastest.  The cache of the benchmark's ensemble is committed with the package
(tuned/launch_shapes.json); bench.py reads it.
"""
from __future__ import annotations

import hashlib
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


def batch_key(domains: list, prec: str) -> str:
    """Cache key of a set of domains: precision, count, a digest of their
    shapes and solid masks, and the digest of the step's source (a timing
    taken with another kernel does not carry over)."""
    from .build import source_digest
    h = hashlib.sha256(prec.encode())
    for d in domains:
        h.update(repr(tuple(d["shape"])).encode())
        h.update(np.ascontiguousarray(d["solid"], dtype=np.uint8).tobytes())
    return f"batch:{prec}:{len(domains)}:{h.hexdigest()[:16]}:{source_digest()}"


def _time_batch(lbm, prec, domains, tile, zchunk, steps, warmup):
    """Seconds per batched step of the domains at one tile shape (None if the
    tile is not compiled for this precision or does not fit a domain)."""
    import time

    import torch
    ctxs = []
    try:
        for d in domains:
            nz, ny, nx = d["shape"]
            ctxs.append(lbm.lbm_init(lbm.Params(nx, ny, nz, prec=lbm.PRECISIONS[prec], solid=d["solid"],
                                                rho_init=(d["rho_A"], d["rho_B"]), tau=d["tau"], G=d["G"], g=d["g"],
                                                rho_s=d["rho_s"], tile=tile, zchunk=zchunk)))
    except lbm.LBMError as e:
        if e.code == lbm.LBM_EINVAL:
            return None
        raise
    b = lbm.lbm_batch_create(ctxs)
    lbm.lbm_batch_step(b, warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lbm.lbm_batch_step(b, steps)   # returns when the work is done
    dt = (time.perf_counter() - t0) / steps
    lbm.lbm_batch_free(b)
    for c in ctxs:
        lbm.lbm_free(c)
    return dt


def tune_batch(domains: list, prec: str = "fp32", steps: int = 16, warmup: int = 4, cache: str | None = None,
               tiles=((64, 8), (64, 16), (32, 16), (32, 8)), zchunks=(0, 32)) -> dict:
    """The launch shape of a batch: every (tile, z-chunk) candidate is timed
    on the whole batch (one launch per step over all domains' tiles, as
    lbm_batch_step runs it) and the fastest kept; z-chunk 0 is each
    context's default.  Cached under batch_key(domains, prec)."""
    from . import lbm
    lbm.load_library()
    key = batch_key(domains, prec)
    table = _load(cache)
    if key in table:
        return table[key]
    times = {}
    for tile in tiles:
        for zc in zchunks:
            t = _time_batch(lbm, prec, domains, tile, zc, steps, warmup)
            if t is not None:
                times[f"{tile[0]}x{tile[1]}/{zc}"] = t * 1e3
    best = min(times, key=times.get)
    tile, zc = best.split("/")
    res = {"tile": [int(v) for v in tile.split("x")], "zchunk": int(zc), "ms": times[best], "all_ms": times,
           "domains": len(domains), "prec": prec}
    table[key] = res
    _save(cache, table)
    return res


def cached_batch_shape(domains: list, prec: str, cache: str):
    """The cached launch shape of this batch, or None if it was never tuned."""
    return _load(cache).get(batch_key(domains, prec))


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
