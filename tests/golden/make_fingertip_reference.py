"""Writes fingertip50k_oracle.npz: FP64 oracle displacements of complete
100-step indentation jobs on the 50k-tet synthetic fingertip.

Only the oracle and the seeded input generators are used (no device code).
Seeds 3000..3003 are the first jobs of the batched benchmark. Saved per seed:
u after load steps 50 and 100, the contact resultant at step 100, and the
oracle's iteration counts. Tolerances: Newton 2e-9 relative (the FP64 gradient
floor on this mesh is ~5e-10 relative to the step's first residual), CG 1e-10.

Run from the repository root:  python tests/golden/make_fingertip_reference.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2103_16747_amd import workload as W  # noqa: E402

SEEDS = (3000, 3001, 3002, 3003)
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fingertip50k_oracle.npz")


def main():
    mesh = W.fingertip_mesh(50000)
    orc = oracle.Solver(mesh.X, mesh.tets, mesh.fixed, E=0.3e6, nu=0.45)
    prm = oracle.default_params(newton_rtol=2e-9, cg_rtol=1e-10)
    data = {"seeds": np.array(SEEDS), "n": mesh.n, "m": mesh.m}
    for seed in SEEDS:
        ind = W.seat_on_mesh(W.random_indentation(seed), mesh)
        t0 = time.time()
        res = orc.solve_indentation(ind, params=prm)
        u50, u100 = res[49][0], res[99][0]
        orc.set_indenter(ind.kind, ind.shape, ind.R, ind.center(ind.steps), ind.k_penalty)
        Ft = orc.contact_patch(u100)[3]
        data[f"u50_{seed}"] = u50
        data[f"u100_{seed}"] = u100
        data[f"F_{seed}"] = Ft
        data[f"status_{seed}"] = np.array([r[1]["status"] for r in res])
        data[f"cg_{seed}"] = np.array([r[1]["cg_iters"] for r in res])
        print(f"seed {seed} {W.KIND_NAMES[ind.kind]} depth {ind.depth*1e3:.2f} mm: {time.time()-t0:.0f} s, "
              f"max|u| {np.abs(u100).max():.3e}, F {Ft}, failed steps {int(np.sum(data[f'status_{seed}'] != 0))}",
              flush=True)
    np.savez_compressed(OUT, **data)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
