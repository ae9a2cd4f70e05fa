"""Full-size parity: complete 100-step indentation jobs on the 50k-tet
fingertip, run as one batch in the benchmark's launch configuration, against
stored FP64 oracle results (tests/golden/fingertip50k_oracle.npz, written by
tests/golden/make_fingertip_reference.py from the oracle alone).

Bounds: e_inf = max_i |u_i - u_i^ref| / max_i |u_i^ref| at load steps 50 and
100 <= 1e-8 on the FP64 path (solves converged to 2e-9 relative residual on
both sides) and <= 1e-4 on the FP32 path at its default tolerances (the
mixed-precision target); the contact resultant at step 100 within 1e-8
(FP64) and 1e-4 (FP32) of the oracle's, relative to its magnitude. Jobs
whose oracle solve reported a failed load step are compared only up to the
last step before it.
"""
import os

import numpy as np
import pytest

from paper_2103_16747_amd import fem, workload as W

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden", "fingertip50k_oracle.npz")


def e_inf(u, ref):
    return float(np.abs(u - ref).max() / max(np.abs(ref).max(), 1e-300))


@pytest.fixture(scope="module")
def gold():
    if not os.path.exists(GOLD):
        pytest.skip("oracle reference file not generated")
    return np.load(GOLD)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_fingertip_jobs_match_oracle(gold, precision):
    mesh = W.fingertip_mesh(50000)
    assert int(gold["n"]) == mesh.n and int(gold["m"]) == mesh.m
    seeds = [int(s) for s in gold["seeds"]]
    checks = []
    for seed in seeds:
        status = gold[f"status_{seed}"]
        ok_until = int(np.argmax(status != 0)) if np.any(status != 0) else len(status)
        for step in (50, 100):
            if step <= ok_until:
                checks.append((seed, step))
    batch = fem.FemBatch(len(seeds), precision)
    mid = batch.add_mesh(mesh.X, mesh.tets, mesh.fixed)
    P = batch.default_params(newton_rtol=2e-9, cg_rtol=1e-10) if precision == "fp64" else batch.default_params()
    inds = {s: W.seat_on_mesh(W.random_indentation(s), mesh) for s in seeds}
    # Run to step 50, compare, then on to step 100.
    for step in (50, 100):
        for s in seeds:
            ind = inds[s]
            half = W.Indentation(ind.kind, ind.shape, ind.R, ind.c0, ind.direction, ind.depth * step / 100.0,
                                 step, ind.k_penalty, seed=s)
            if step == 50:
                batch.add_job(mid, half)
        if step == 50:
            assert batch.run(P) == 0
            u50 = {s: batch.displacements(j) for j, s in enumerate(seeds)}
    # Full jobs in a fresh batch (same launch configuration as the benchmark).
    full = fem.FemBatch(len(seeds), precision)
    fmid = full.add_mesh(mesh.X, mesh.tets, mesh.fixed)
    ids = {s: full.add_job(fmid, inds[s]) for s in seeds}
    assert full.run(P) == 0
    bound = 1e-8 if precision == "fp64" else 1e-4
    for seed, step in checks:
        u = u50[seed] if step == 50 else full.displacements(ids[seed])
        err = e_inf(u, gold[f"u{step}_{seed}"])
        print(f"{precision} seed {seed} step {step}: e_inf {err:.3e}", flush=True)
        assert err <= bound, (seed, step, err)
        if step == 100:
            Ft = full.contact_patch(ids[seed])[3]
            Fr = gold[f"F_{seed}"]
            ef = float(np.abs(Ft - Fr).max() / max(np.abs(Fr).max(), 1e-300))
            print(f"{precision} seed {seed} resultant {Ft} oracle {Fr}: rel err {ef:.3e}", flush=True)
            assert ef <= bound, (seed, Ft, Fr)
    batch.close()
    full.close()


DYN_GOLD = os.path.join(os.path.dirname(__file__), "golden", "fingertip50k_dynamic_oracle.npz")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_fingertip_time_steps_match_oracle(precision):
    """Backward-Euler time steps (dt = 1e-4 s) of the benchmark's first jobs
    on the 50k fingertip, batched, against stored oracle results
    (tests/golden/make_fingertip_dynamic_reference.py): displacements within
    1e-8 (FP64) and 1e-4 (FP32), velocities within 10x those bounds (a
    velocity is a difference of displacements over dt)."""
    if not os.path.exists(DYN_GOLD):
        pytest.skip("oracle reference file not generated")
    gold = np.load(DYN_GOLD)
    mesh = W.fingertip_mesh(50000)
    steps, dt, rho = int(gold["steps"]), float(gold["dt"]), float(gold["rho"])
    seeds = [int(s) for s in gold["seeds"]]
    batch = fem.FemBatch(len(seeds), precision)
    mid = batch.add_mesh(mesh.X, mesh.tets, mesh.fixed)
    ids = {}
    for s in seeds:
        ind = W.seat_on_mesh(W.random_indentation(s), mesh)
        short = W.Indentation(ind.kind, ind.shape, ind.R, ind.c0, ind.direction, ind.depth * steps / ind.steps, steps,
                              ind.k_penalty, dt=dt, density=rho)
        ids[s] = batch.add_job(mid, short)
    P = batch.default_params(newton_rtol=2e-9, cg_rtol=1e-10) if precision == "fp64" else batch.default_params()
    assert batch.run(P) == 0
    bound = 1e-8 if precision == "fp64" else 1e-4
    for s in seeds:
        eu = e_inf(batch.displacements(ids[s]), gold[f"u_{s}"])
        ev = e_inf(batch.velocities(ids[s]), gold[f"v_{s}"])
        print(f"{precision} dynamic seed {s} step {steps}: e_inf u {eu:.3e} v {ev:.3e}", flush=True)
        assert eu <= bound and ev <= 10 * bound, (s, eu, ev)
    batch.close()
