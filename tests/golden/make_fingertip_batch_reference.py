"""Writes the FP64 oracle references of the 256-job fingertip batch
(50k-tet synthetic fingertip, seeds 3000..3255, 100 quasi-static load steps
each):

- fingertip50k_batch_summary.npz: for EVERY seed and load step, the oracle's
  status, Newton and CG iteration counts, the displacement statistics of the
  paper's Sec. IV (max_i |u_i| and mean_i |u_i|), the contact resultant and
  the number of contact nodes;
- fingertip50k_stratified_oracle.npz: the full displacement field after
  load steps 50 and 100, plus the contact patch (node ids, forces, phi) at
  step 100, of a 16-seed stratified subset (four per indenter kind, chosen by
  the rule in `select`).

Only the oracle and the seeded input generators are used (no device code).
Tolerances: Newton 2e-9 relative (the FP64 gradient floor on this mesh is
about 5e-10 of a step's first residual), CG 1e-10. Per-seed results are
cached under --cache (keyed by seed, mesh hash and tolerances), so an
interrupted run resumes.

Run from the repository root:
    python tests/golden/make_fingertip_batch_reference.py [--workers 7]
"""
import argparse
import hashlib
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2103_16747_amd import workload as W  # noqa: E402

SEEDS = tuple(range(3000, 3256))
NEWTON_RTOL, CG_RTOL = 2e-9, 1e-10
HERE = os.path.dirname(os.path.abspath(__file__))
OUT_SUMMARY = os.path.join(HERE, "fingertip50k_batch_summary.npz")
OUT_STRAT = os.path.join(HERE, "fingertip50k_stratified_oracle.npz")
# Seeds whose FP32 batch run ends at least one load step at the Newton cap;
# they are kept in the subset so that the device's failed steps meet an
# oracle status. Only the choice of seeds comes from the device run, never a
# stored value.
# (A run of the 256-job FP32 batch ended load steps at the Newton cap on
# rings 3017, 3040, 3041, 3053, ..., boxes 3068 (steps 9-18), 3050, 3048, ...
# and cylinder 3156; listed by priority within each kind.)
DEVICE_CAPPED_SEEDS = (3017, 3040, 3068, 3050, 3156)

_mesh = None
_solver = None


def mesh_hash(mesh):
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(mesh.X, dtype=np.float64).tobytes())
    h.update(np.ascontiguousarray(mesh.tets, dtype=np.int32).tobytes())
    h.update(np.ascontiguousarray(mesh.fixed, dtype=np.uint8).tobytes())
    return h.hexdigest()[:16]


def _init():
    global _mesh, _solver
    _mesh = W.fingertip_mesh(50000)
    _solver = oracle.Solver(_mesh.X, _mesh.tets, _mesh.fixed, E=0.3e6, nu=0.45)


def solve_seed(args):
    seed, path = args
    mesh, orc = _mesh, _solver
    prm = oracle.default_params(newton_rtol=NEWTON_RTOL, cg_rtol=CG_RTOL)
    ind = W.seat_on_mesh(W.random_indentation(seed), mesh)
    S = ind.steps
    rec = {k: np.zeros(S, dtype=np.int32) for k in ("status", "newton", "cg", "n_contact")}
    rec.update({"umax": np.zeros(S), "umean": np.zeros(S), "F": np.zeros((S, 3))})
    keep = {}

    def cb(k, u, info):
        i = k - 1
        rec["status"][i], rec["newton"][i], rec["cg"][i] = info["status"], info["newton_iters"], info["cg_iters"]
        rec["umax"][i], rec["umean"][i] = oracle.displacement_stats(u)
        ids, f, phi, Ft = orc.contact_patch(u)     # the indenter of step k is set
        rec["F"][i], rec["n_contact"][i] = Ft, len(ids)
        if k in (50, 100):
            keep[f"u{k}"] = u.copy()
        if k == 100:
            keep["ids100"], keep["f100"], keep["phi100"] = ids, f, phi

    t0 = time.time()
    orc.solve_indentation(ind, params=prm, callback=cb)
    np.savez_compressed(path + ".tmp.npz", kind=ind.kind, depth=ind.depth, **rec, **keep)
    os.replace(path + ".tmp.npz", path)
    return seed, time.time() - t0, int(np.sum(rec["status"] != 0))


def select(summ):
    """Four seeds per indenter kind: the seeds the device's FP32 batch ends
    with a capped step (at most two per kind), then the seeds whose oracle
    solve fails a load step (at most one more), then the deepest job, then
    the most CG work, until four are chosen."""
    chosen = []
    seeds = summ["seeds"]
    for kind in range(4):
        mine = [int(s) for s, k in zip(seeds, summ["kind"]) if k == kind]
        idx = {s: i for i, s in enumerate(seeds.tolist())}
        pick = [s for s in DEVICE_CAPPED_SEEDS if s in mine][:2]
        orc_fail = [s for s in mine if np.any(summ["status"][idx[s]] != 0) and s not in pick]
        pick += orc_fail[:1]
        for s in sorted(mine, key=lambda s: -summ["depth"][idx[s]]):
            if len(pick) >= 3:
                break
            if s not in pick:
                pick.append(s)
        for s in sorted(mine, key=lambda s: -int(summ["cg"][idx[s]].sum())):
            if len(pick) >= 4:
                break
            if s not in pick:
                pick.append(s)
        chosen += pick
    return sorted(chosen)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=max(1, (os.cpu_count() or 2) - 1))
    ap.add_argument("--cache", default=os.path.join("/tmp", "fingertip50k_oracle_cache"))
    a = ap.parse_args()
    mesh = W.fingertip_mesh(50000)
    mh = mesh_hash(mesh)
    cdir = os.path.join(a.cache, f"{mh}_n{NEWTON_RTOL:g}_cg{CG_RTOL:g}")
    os.makedirs(cdir, exist_ok=True)
    todo = [(s, os.path.join(cdir, f"seed_{s}.npz")) for s in SEEDS]
    missing = [t for t in todo if not os.path.exists(t[1])]
    print(f"mesh {mh}: {mesh.n} nodes, {mesh.m} tets; {len(missing)} of {len(SEEDS)} seeds to solve", flush=True)
    if missing:
        with mp.get_context("fork").Pool(a.workers, initializer=_init) as pool:
            for seed, dt, nf in pool.imap_unordered(solve_seed, missing):
                print(f"seed {seed}: {dt:.0f} s, failed steps {nf}", flush=True)
    per = {s: np.load(p) for s, p in todo}
    summ = {"seeds": np.array(SEEDS), "n": mesh.n, "m": mesh.m, "mesh_hash": mh,
            "newton_rtol": NEWTON_RTOL, "cg_rtol": CG_RTOL,
            "kind": np.array([int(per[s]["kind"]) for s in SEEDS]),
            "depth": np.array([float(per[s]["depth"]) for s in SEEDS])}
    for k in ("status", "newton", "cg", "n_contact", "umax", "umean", "F"):
        summ[k] = np.stack([per[s][k] for s in SEEDS])
    np.savez_compressed(OUT_SUMMARY, **summ)
    chosen = select(summ)
    strat = {"seeds": np.array(chosen), "n": mesh.n, "m": mesh.m, "mesh_hash": mh,
             "newton_rtol": NEWTON_RTOL, "cg_rtol": CG_RTOL}
    for s in chosen:
        for k in ("u50", "u100", "ids100", "f100", "phi100"):
            strat[f"{k}_{s}"] = per[s][k]
    np.savez_compressed(OUT_STRAT, **strat)
    fails = {s: int(np.sum(per[s]["status"] != 0)) for s in SEEDS if np.any(per[s]["status"] != 0)}
    print("oracle failed steps per seed:", fails)
    print("stratified subset:", [(s, W.KIND_NAMES[int(per[s]["kind"])], round(float(per[s]["depth"]) * 1e3, 2))
                                 for s in chosen])
    print("wrote", OUT_SUMMARY, "and", OUT_STRAT)


if __name__ == "__main__":
    main()
