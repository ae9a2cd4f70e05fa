"""Writes fingertip50k_dynamic_oracle.npz: FP64 oracle backward-Euler time
steps (dt = 1e-4 s, lumped masses at 1100 kg/m^3) of the first jobs of the
batched benchmark on the 50k-tet synthetic fingertip.

Only the oracle and the seeded input generators are used (no device code).
Saved per seed: u and v after STEPS time steps, and the oracle's status per
step. Tolerances: Newton 2e-9 relative, CG 1e-10.

Run from the repository root:  python tests/golden/make_fingertip_dynamic_reference.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2103_16747_amd import workload as W  # noqa: E402

SEEDS = (3000, 3001)
STEPS = 10
DT, RHO = 1e-4, 1100.0
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fingertip50k_dynamic_oracle.npz")


def main():
    mesh = W.fingertip_mesh(50000)
    orc = oracle.Solver(mesh.X, mesh.tets, mesh.fixed, E=0.3e6, nu=0.45)
    prm = oracle.default_params(newton_rtol=2e-9, cg_rtol=1e-10)
    data = {"seeds": np.array(SEEDS), "n": mesh.n, "m": mesh.m, "steps": STEPS, "dt": DT, "rho": RHO}
    for seed in SEEDS:
        ind = W.seat_on_mesh(W.random_indentation(seed), mesh)
        t0 = time.time()
        res = orc.solve_dynamic(ind, DT, RHO, params=prm, steps=STEPS)
        data[f"u_{seed}"] = res[-1][0]
        data[f"v_{seed}"] = res[-1][1]
        data[f"status_{seed}"] = np.array([r[2]["status"] for r in res])
        print(f"seed {seed}: {time.time() - t0:.1f} s, statuses {set(int(r[2]['status']) for r in res)}", flush=True)
    np.savez_compressed(OUT, **data)


if __name__ == "__main__":
    main()
