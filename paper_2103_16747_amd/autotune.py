"""Autotuner for the batched engine's shape parameters, per mesh-size class.

Per mesh, the tile shape (tets per tile and distinct nodes per tile) trades
per-block work and LDS occupancy against tile-entry duplication (the halo:
gather and partial-write traffic of nodes shared by tiles); the best shape
depends on the mesh's size and element grading, so each mesh of a mix is
tuned on its own: a short batched run of seeded jobs on that mesh alone for
every candidate shape, the fastest per tet-update kept. For the whole mix,
the round length (solver steps between host polls) trades idle steps of
finished jobs against round overheads; it is tuned last, with the per-mesh
shapes applied. The per-mesh results are cached in a JSON file keyed by
(mesh hash, precision), the round length by the mix's key, so a known mesh
is never re-timed.
"""
from __future__ import annotations

import hashlib
import json
import os
import time

import numpy as np

from . import fem, workload as W

# (tets per tile, distinct nodes per tile); the library's limits are
# 64..512 tets and 16..256 nodes (8-bit local slots)
SHAPE_CANDIDATES = ((512, 256), (384, 256), (256, 256), (256, 128), (128, 128))
CHUNK_CANDIDATES = (8, 16, 32, 64)


def mesh_key(mesh, precision):
    """Cache key of one mesh: a hash of its nodes, tets and fixed mask, and
    the precision."""
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(mesh.X, dtype=np.float64).tobytes())
    h.update(np.ascontiguousarray(mesh.tets, dtype=np.int32).tobytes())
    h.update(np.ascontiguousarray(mesh.fixed, dtype=np.uint8).tobytes())
    return f"{precision}:{h.hexdigest()[:16]}"


def _short_jobs(mesh, count, seed0, steps):
    return [W.seat_on_mesh(W.random_indentation(seed0 + i, steps=steps), mesh) for i in range(count)]


def _time_config(meshes, jobs, precision, shapes, chunk):
    """Wall time and tet-updates of one warm run of `jobs` (a list per mesh)
    with the given tile shape per mesh and round length."""
    batch = fem.FemBatch(sum(len(j) for j in jobs), precision)
    batch.set_option(fem.FEM_OPT_ROUND_STEPS, chunk)
    mids = []
    for m, (tets, nodes) in zip(meshes, shapes):
        batch.set_option(fem.FEM_OPT_TILE_TETS, tets)
        batch.set_option(fem.FEM_OPT_TILE_NODES, nodes)
        mids.append(batch.add_mesh(m.X, m.tets, m.fixed))
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


def _load(cache):
    if cache and os.path.exists(cache):
        with open(cache) as f:
            return json.load(f)
    return {}


def _store(cache, known):
    if cache:
        tmp = cache + ".tmp"
        with open(tmp, "w") as f:
            json.dump(known, f, indent=1)
        os.replace(tmp, cache)


def tune_mesh(mesh, precision="fp32", jobs=16, steps=4, seed0=7000, cache=None, log=None):
    """Tile shape for one mesh: {"tile_tets", "tile_nodes", "table"}, the
    candidate with the most tet-updates per second on a short run of `jobs`
    seeded jobs of `steps` load steps (round length 16)."""
    key = mesh_key(mesh, precision)
    known = _load(cache)
    if key in known.get("meshes", {}):
        return known["meshes"][key]
    js = [_short_jobs(mesh, jobs, seed0, steps)]
    table = []
    for tets, nodes in SHAPE_CANDIDATES:
        wall, tu = _time_config([mesh], js, precision, [(tets, nodes)], 16)
        table.append({"tile_tets": tets, "tile_nodes": nodes, "wall_s": wall, "tet_updates_per_s": tu / wall})
        if log:
            log(f"autotune {mesh.m}-tet mesh: tile {tets} tets / {nodes} nodes: {tu / wall:.3e} tet-updates/s")
    best = max(table, key=lambda r: r["tet_updates_per_s"])
    out = {"tets": mesh.m, "tile_tets": best["tile_tets"], "tile_nodes": best["tile_nodes"], "table": table}
    known = _load(cache)
    known.setdefault("meshes", {})[key] = out
    _store(cache, known)
    return out


def tune(meshes, precision="fp32", jobs_per_mesh=4, steps=4, seed0=7000, cache=None, log=None):
    """Shapes for a mix of meshes: per mesh its tuned tile shape
    (tune_mesh), then the round length for the mix with those shapes on a
    short run of jobs_per_mesh jobs per mesh. Returns {"shapes": [(tile_tets,
    tile_nodes) per mesh], "chunk", "per_mesh": [...], "table": [...]}."""
    per = [tune_mesh(m, precision, seed0=seed0 + 1000 * i, cache=cache, log=log) for i, m in enumerate(meshes)]
    shapes = [(p["tile_tets"], p["tile_nodes"]) for p in per]
    mix = f"{precision}:" + ",".join(mesh_key(m, precision).split(":")[1] for m in meshes)
    known = _load(cache)
    if mix in known.get("mixes", {}):
        chunk, table = known["mixes"][mix]["chunk"], known["mixes"][mix]["table"]
    else:
        jobs = [_short_jobs(m, jobs_per_mesh, seed0 + 100 * i, steps) for i, m in enumerate(meshes)]
        table = []
        for c in CHUNK_CANDIDATES:
            wall, tu = _time_config(meshes, jobs, precision, shapes, c)
            table.append({"chunk": c, "wall_s": wall, "tet_updates_per_s": tu / wall})
            if log:
                log(f"autotune mix: round length {c}: {wall * 1e3:.1f} ms")
        chunk = min(table, key=lambda r: r["wall_s"])["chunk"]
        known = _load(cache)
        known.setdefault("mixes", {})[mix] = {"chunk": chunk, "table": table}
        _store(cache, known)
    return {"shapes": shapes, "chunk": chunk, "per_mesh": per, "table": table}


def apply_shape(batch, shape):
    """Sets the tile limits for the next mesh added to `batch`."""
    batch.set_option(fem.FEM_OPT_TILE_TETS, shape[0])
    batch.set_option(fem.FEM_OPT_TILE_NODES, shape[1])
