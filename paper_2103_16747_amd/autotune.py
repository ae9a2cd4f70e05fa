"""Autotuner for the batched engine's shape parameters.

Two shapes matter for a batch: the tile size (tets per tile, which trades LDS
reuse and per-block work against tile-entry duplication, i.e. gather and
partial-write traffic) and the CG chunk (iterations per round, which trades
idle iterations of jobs whose CG has finished against round overheads). The
tuner times a short batched run of the caller's mesh mix for each candidate
and returns the fastest; results can be cached in a JSON file keyed by the
mesh sizes and precision.
"""
from __future__ import annotations

import json
import os
import time

from . import fem, workload as W

TILE_CANDIDATES = (256, 512)
CHUNK_CANDIDATES = (8, 16, 32)


def _short_jobs(mesh, count, seed0, steps):
    out = []
    for i in range(count):
        ind = W.seat_on_mesh(W.random_indentation(seed0 + i, steps=steps), mesh)
        out.append(ind)
    return out


def _time_config(meshes, jobs, precision, tile, chunk):
    batch = fem.FemBatch(sum(len(j) for j in jobs), precision)
    batch.set_option(fem.FEM_OPT_TILE_TETS, tile)
    batch.set_option(fem.FEM_OPT_ROUND_STEPS, chunk)
    mids = [batch.add_mesh(m.X, m.tets, m.fixed) for m in meshes]
    ids = [(batch.add_job(mid, ind), ind) for mid, js in zip(mids, jobs) for ind in js]
    batch.run()                       # warm-up: graphs captured, caches warm
    for j, ind in ids:
        batch.restart_job(j, ind)
    t0 = time.perf_counter()
    batch.run()
    wall = time.perf_counter() - t0
    tu = sum(batch.job_info(j)["tet_updates"] for j, _ in ids)
    batch.close()
    return wall, tu


def tune(meshes, precision="fp32", jobs_per_mesh=4, steps=4, seed0=7000, cache=None, log=None):
    """Returns {"tile_tets", "chunk", "table"} for the fastest candidate on a
    short run (jobs_per_mesh seeded jobs of `steps` load steps per mesh)."""
    key = f"{precision}:" + ",".join(str(m.m) for m in meshes)
    if cache and os.path.exists(cache):
        with open(cache) as f:
            known = json.load(f)
        if key in known:
            return known[key]
    jobs = [_short_jobs(m, jobs_per_mesh, seed0 + 100 * i, steps) for i, m in enumerate(meshes)]
    table = []
    for tile in TILE_CANDIDATES:
        for chunk in CHUNK_CANDIDATES:
            wall, tu = _time_config(meshes, jobs, precision, tile, chunk)
            table.append({"tile_tets": tile, "chunk": chunk, "wall_s": wall, "tet_updates_per_s": tu / wall})
            if log:
                log(f"autotune tile {tile} chunk {chunk}: {wall * 1e3:.1f} ms")
    best = min(table, key=lambda r: r["wall_s"])
    out = {"tile_tets": best["tile_tets"], "chunk": best["chunk"], "table": table}
    if cache:
        known = {}
        if os.path.exists(cache):
            with open(cache) as f:
                known = json.load(f)
        known[key] = out
        with open(cache, "w") as f:
            json.dump(known, f, indent=1)
    return out
