"""Parity of implicit (backward-Euler) time steps on the HIP path against the
FP64 oracle (runs on an MI355X).

A step minimises Pi(u) + sum_i m_i/(2 dt^2)|u_i - ut_i|^2 with lumped masses,
ut = u^n + dt v^n, then v^{n+1} = (u^{n+1} - u^n)/dt. Tolerances as for the
quasi-static solves: e_inf <= 1e-8 on the FP64 path (both sides converged to
1e-10 relative residual), <= 1e-4 on the FP32 path; velocities are compared
relative to their largest entry with the same bounds times 10 (a velocity is
a difference of two displacements over dt).
"""
import numpy as np
import pytest

from paper_2103_16747_amd import fem, workload as W

pytestmark = pytest.mark.gpu

E0, NU0, RHO = 0.3e6, 0.45, 1100.0


def say(*a):
    print(*a, flush=True)


def e_inf(u, ref):
    return float(np.abs(u - ref).max() / max(np.abs(ref).max(), 1e-300))


def params(obj, precision):
    if precision == "fp64":
        return obj.default_params(newton_rtol=1e-10, cg_rtol=1e-10)
    return obj.default_params()


BOUND = {"fp64": 1e-8, "fp32": 1e-4}


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("dt", [1e-4, 1e-3])
def test_cube_time_steps_match_oracle(oracle_lib, precision, dt):
    """The cube and sphere schedule as time steps of dt: the indenter moves
    0.15 mm per step, so at 1e-4 s inertia dominates the first steps."""
    say("case cube dynamic", precision, dt)
    mesh = W.cube_block_mesh()
    ind = W.cube_sphere_indentation()
    orc = oracle_lib.Solver(mesh.X, mesh.tets, mesh.fixed, E=E0, nu=NU0)
    ref = orc.solve_dynamic(ind, dt, RHO, params=oracle_lib.default_params(newton_rtol=1e-11, cg_rtol=1e-11))
    dev = fem.FemMesh(mesh.X, mesh.tets, mesh.fixed, precision=precision)
    dev.set_material(E0, NU0, RHO)
    dev.set_dynamics(dt)
    P = params(dev, precision)
    worst_u = worst_v = 0.0
    for k in range(1, ind.steps + 1):
        dev.set_indenter(ind.kind, ind.shape, ind.R, ind.center(k), ind.k_penalty)
        info = dev.step(P)
        assert info["status"] >= 0, (k, info)
        u_ref, v_ref, _ = ref[k - 1]
        worst_u = max(worst_u, e_inf(dev.displacements(), u_ref))
        worst_v = max(worst_v, e_inf(dev.velocities(), v_ref))
        say(k, info["newton_iters"], info["cg_iters"], "e_inf u %.3e v %.3e" % (worst_u, worst_v))
    assert worst_u <= BOUND[precision]
    assert worst_v <= 10 * BOUND[precision]
    dev.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_free_body_translates_with_its_velocity(precision):
    """No fixed nodes, no contact: a uniform initial velocity carries the body
    dt v per step, and the velocity is kept."""
    mesh = W.block_mesh((2, 2, 3), (2e-3, 2e-3, 3e-3))
    dev = fem.FemMesh(mesh.X, mesh.tets, np.zeros(mesh.n, dtype=np.uint8), precision=precision)
    dev.set_material(E0, NU0, RHO)
    dev.set_indenter(W.SPHERE, [1e-3], np.eye(3), [1.0, 1.0, 1.0])
    dt = 1e-4
    dev.set_dynamics(dt)
    v0 = np.tile([0.1, -0.2, 0.05], (mesh.n, 1))
    dev.set_velocities(v0)
    for k in range(1, 6):
        info = dev.step(params(dev, precision))
        assert info["status"] >= 0, info
        assert e_inf(dev.displacements(), k * dt * v0) <= BOUND[precision]
        assert e_inf(dev.velocities(), v0) <= 10 * BOUND[precision]
    dev.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batched_time_steps_match_oracle(oracle_lib, precision):
    """Fingertip (5k tets) jobs as time steps in one batch, with a
    quasi-static job beside them; each against its own oracle run."""
    mesh = W.fingertip_mesh(5000)
    jobs = []
    for s, dt in ((4200, 1e-4), (4201, 2e-4), (4202, 0.0)):
        ind = W.seat_on_mesh(W.random_indentation(s, steps=8), mesh)
        ind.dt = dt
        ind.density = RHO
        jobs.append(ind)
    batch = fem.FemBatch(len(jobs), precision)
    mid = batch.add_mesh(mesh.X, mesh.tets, mesh.fixed)
    ids = [batch.add_job(mid, j, E0, NU0) for j in jobs]
    assert batch.run(params(batch, precision)) == 0
    P = oracle_lib.default_params(newton_rtol=1e-11, cg_rtol=1e-11)
    for jid, job in zip(ids, jobs):
        info = batch.job_info(jid)
        assert info["done"] == 1 and info["status"] == 0, info
        orc = oracle_lib.Solver(mesh.X, mesh.tets, mesh.fixed, E=E0, nu=NU0)
        if job.dt > 0:
            u_ref, v_ref, _ = orc.solve_dynamic(job, job.dt, RHO, params=P)[-1]
        else:
            u_ref, _ = orc.solve_indentation(job, params=P)[-1]
            v_ref = np.zeros_like(u_ref)
        eu = e_inf(batch.displacements(jid), u_ref)
        v = batch.velocities(jid)
        ev = e_inf(v, v_ref) if job.dt > 0 else float(np.abs(v).max())
        say(job.seed, job.dt, "e_inf u %.3e v %.3e" % (eu, ev), "newton", info["newton_iters"], "cg", info["cg_iters"])
        assert eu <= BOUND[precision]
        assert ev <= (10 * BOUND[precision] if job.dt > 0 else 0.0)
    batch.close()
