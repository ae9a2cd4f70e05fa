"""Parity of the co-rotational law on the HIP path against the FP64 oracle
(runs on an MI355X).

Co-rotational linear elasticity is the constitutive model of the paper's own
simulator (Sec. III-A), with its calibrated E = 1.55 MPa, nu = 0.316. The same
tolerances as the Neo-Hookean parity tests: single evaluations 1e-11 (FP64)
and 2e-5 (FP32) relative to the largest entry; solves e_inf <= 1e-8 (FP64,
both sides converged to 1e-10 relative residual) and <= 1e-4 (FP32).
"""
import numpy as np
import pytest

from paper_2103_16747_amd import fem, workload as W
from test_gpu_parity import indenter_for

pytestmark = pytest.mark.gpu

E_G, NU_G = 1.55e6, 0.316
E0, NU0 = 0.3e6, 0.45
SINGLE = {"fp64": 1e-11, "fp32": 2e-5}
SOLVE = {"fp64": 1e-8, "fp32": 1e-4}


def say(*a):
    print(*a, flush=True)


def e_inf(u, ref):
    return float(np.abs(u - ref).max() / max(np.abs(ref).max(), 1e-300))


def make_pair(oracle_lib, mesh, precision, ind=None, center=None):
    dev = fem.FemMesh(mesh.X, mesh.tets, mesh.fixed, precision=precision)
    dev.set_material(E_G, NU_G, 1100.0)
    dev.set_model(fem.FEM_MODEL_COROTATIONAL)
    orc = oracle_lib.Solver(mesh.X, mesh.tets, mesh.fixed, E=E_G, nu=NU_G)
    orc.set_model(oracle_lib.COROTATIONAL)
    if ind is not None:
        c = ind.center(1) if center is None else center
        dev.set_indenter(ind.kind, ind.shape, ind.R, c, ind.k_penalty)
        orc.set_indenter(ind.kind, ind.shape, ind.R, c, ind.k_penalty)
    return dev, orc


MESHES = {
    "cube8": lambda: W.cube_block_mesh(),
    "fingertip5k": lambda: W.fingertip_mesh(5000),
    "fingertip50k": lambda: W.fingertip_mesh(50000),
}


@pytest.fixture(scope="module")
def meshes():
    return {k: f() for k, f in MESHES.items()}


@pytest.mark.parametrize("name", list(MESHES))
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_gradient_and_energy_parity(oracle_lib, meshes, name, precision):
    say("case corotational gradient", name, precision)
    mesh = meshes[name]
    ind = indenter_for(mesh, W.SPHERE, 300)
    dev, orc = make_pair(oracle_lib, mesh, precision, ind, center=ind.c0)
    u = W.random_displacement(mesh, 31, 0.01)
    if precision == "fp32":
        u = u.astype(np.float32).astype(np.float64)
    dev.set_displacements(u)
    g, e, mj = dev.gradient()
    g_ref = orc.gradient(u)
    e_ref, mj_ref = orc.energy(u)
    tol = SINGLE[precision]
    err = np.abs(g - g_ref).max() / np.abs(g_ref).max()
    say("gradient e %.3e energy e %.3e" % (err, abs(e - e_ref) / abs(e_ref)))
    assert err <= tol
    assert e == pytest.approx(e_ref, rel=tol * 10)
    assert mj == pytest.approx(mj_ref, rel=tol * 10)
    dev.close()


@pytest.mark.parametrize("name", ["cube8", "fingertip50k"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_hessvec_parity(oracle_lib, meshes, name, precision):
    """The exact tangent, the rotation derivative included."""
    say("case corotational hessvec", name, precision)
    mesh = meshes[name]
    ind = indenter_for(mesh, W.SPHERE, 301)
    dev, orc = make_pair(oracle_lib, mesh, precision, ind, center=ind.c0)
    u = W.random_displacement(mesh, 32, 0.01)
    v = np.random.default_rng(33).normal(size=u.shape)
    if precision == "fp32":
        u = u.astype(np.float32).astype(np.float64)
        v = v.astype(np.float32).astype(np.float64)
    dev.set_displacements(u)
    q = dev.hessvec(v, dev.default_params(contact_hessian=1))
    q_ref = orc.hessvec(u, v, contact_full=1)
    err = np.abs(q - q_ref).max() / np.abs(q_ref).max()
    say("hessvec e %.3e" % err)
    assert err <= SINGLE[precision]
    dev.close()


def tight(dev, precision):
    if precision == "fp64":
        return dev.default_params(newton_rtol=1e-10, cg_rtol=1e-10)
    return dev.default_params()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_cube_indentation_parity(oracle_lib, meshes, precision):
    say("case corotational cube indentation", precision)
    mesh = meshes["cube8"]
    ind = W.cube_sphere_indentation()
    dev, orc = make_pair(oracle_lib, mesh, precision)
    ref = orc.solve_indentation(ind, params=oracle_lib.default_params(newton_rtol=1e-11, cg_rtol=1e-11))
    P = tight(dev, precision)
    worst = 0.0
    for k in range(1, ind.steps + 1):
        dev.set_indenter(ind.kind, ind.shape, ind.R, ind.center(k), ind.k_penalty)
        info = dev.step(P)
        assert info["status"] >= 0, (k, info)
        worst = max(worst, e_inf(dev.displacements(), ref[k - 1][0]))
        say(k, info["newton_iters"], info["cg_iters"], "e_inf %.3e" % worst)
    assert worst <= SOLVE[precision]
    sig, vm = dev.tet_stress()
    sig_ref, vm_ref = orc.tet_stress(ref[-1][0])
    scale = np.abs(sig_ref).max()
    assert np.abs(sig - sig_ref).max() <= 10 * SOLVE[precision] * scale
    assert np.abs(vm - vm_ref).max() <= 10 * SOLVE[precision] * scale
    dev.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_tet_stress_at_a_given_state(oracle_lib, meshes, precision):
    say("case corotational tet stress", precision)
    mesh = meshes["fingertip50k"]
    dev, orc = make_pair(oracle_lib, mesh, precision)
    u = W.random_displacement(mesh, 34, 5e-4)
    dev.set_displacements(u)
    sig, vm = dev.tet_stress()
    sig_ref, vm_ref = orc.tet_stress(u)
    scale = np.abs(sig_ref).max()
    err = max(np.abs(sig - sig_ref).max(), np.abs(vm - vm_ref).max()) / scale
    say("stress e %.3e" % err)
    assert err <= SINGLE[precision]
    dev.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_fingertip_first_steps_parity(oracle_lib, meshes, precision):
    """Full-size fingertip (50k tets), seeded indenters, first load steps taken
    at 10x the nominal increment."""
    mesh = meshes["fingertip50k"]
    for seed in (2001, 2004):
        say("case corotational fingertip", precision, seed)
        ind = W.seat_on_mesh(W.random_indentation(seed, steps=10), mesh)
        dev, orc = make_pair(oracle_lib, mesh, precision)
        ref = orc.solve_indentation(ind, steps=3, params=oracle_lib.default_params(newton_rtol=1e-11, cg_rtol=1e-11))
        P = tight(dev, precision)
        for k in range(1, 4):
            dev.set_indenter(ind.kind, ind.shape, ind.R, ind.center(k), ind.k_penalty)
            info = dev.step(P)
            assert info["status"] >= 0, (k, info)
            err = e_inf(dev.displacements(), ref[k - 1][0])
            say(seed, k, info["newton_iters"], info["cg_iters"], "e_inf %.3e" % err)
            assert err <= SOLVE[precision]
        dev.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_mixed_law_batch(oracle_lib, meshes, precision):
    """Neo-Hookean and co-rotational jobs in one batch, one of them with
    implicit time steps; each against its own oracle run. Job 4400 presses a
    box 2.8 mm into the 3 mm skin: without the Neo-Hookean ln J barrier the
    co-rotational law lets elements invert, and the oracle's last load step
    fails with an inverted element; the device reports the same failure for
    that job at that load step, and the same job stopped at 5/6 of its
    depth is compared."""
    mesh = meshes["fingertip5k"]
    spec = [(4400, 1, E_G, NU_G, 0.0, 6), (4400, 1, E_G, NU_G, 0.0, 5), (4401, 0, E0, NU0, 0.0, 6),
            (4402, 1, E_G, NU_G, 2e-4, 6), (4403, 0, E0, NU0, 0.0, 6), (4404, 1, E_G, NU_G, 0.0, 6)]
    jobs = []
    for seed, model, E, nu, dt, steps in spec:
        ind = W.seat_on_mesh(W.random_indentation(seed, steps=6), mesh)
        ind = W.Indentation(ind.kind, ind.shape, ind.R, ind.c0, ind.direction, ind.depth * steps / 6, steps,
                            ind.k_penalty, seed=seed, dt=dt, model=model)
        jobs.append((ind, E, nu))
    batch = fem.FemBatch(len(jobs), precision)
    mid = batch.add_mesh(mesh.X, mesh.tets, mesh.fixed)
    ids = [batch.add_job(mid, ind, E, nu) for ind, E, nu in jobs]
    assert batch.run(tight(batch, precision)) == 0
    P = oracle_lib.default_params(newton_rtol=1e-11, cg_rtol=1e-11)
    for jid, (ind, E, nu) in zip(ids, jobs):
        info = batch.job_info(jid)
        orc = oracle_lib.Solver(mesh.X, mesh.tets, mesh.fixed, E=E, nu=nu)
        orc.set_model(ind.model)
        if ind.dt > 0:
            ref = [(u, i) for u, v, i in orc.solve_dynamic(ind, ind.dt, ind.density, params=P)]
        else:
            ref = orc.solve_indentation(ind, params=P)
        failed = [i["status"] for _, i in ref if i["status"] < 0]
        say(ind.seed, ind.model, ind.dt, ind.steps, "status", info["status"], "oracle failures", failed)
        assert info["done"] == 1
        if failed:
            # the failing step is the same; which limit ends it (inversion
            # or the Newton cap) may differ with the rounding
            assert info["status"] < 0 and info["steps_failed"] == len(failed)
            continue
        assert info["status"] >= 0, info
        err = e_inf(batch.displacements(jid), ref[-1][0])
        say("e_inf %.3e" % err, "newton", info["newton_iters"], "cg", info["cg_iters"])
        assert err <= SOLVE[precision]
    batch.close()


def test_model_is_validated():
    mesh = W.block_mesh((1, 1, 1), (2e-3, 2e-3, 2e-3))
    dev = fem.FemMesh(mesh.X, mesh.tets, mesh.fixed, precision="fp32")
    with pytest.raises(fem.FemError):
        dev.set_model(2)
    dev.close()
    ind = W.seat_on_mesh(W.random_indentation(4405, steps=2), W.fingertip_mesh(5000))
    ind.model = 5
    batch = fem.FemBatch(1, "fp32")
    mid = batch.add_mesh(mesh.X, mesh.tets, mesh.fixed)
    with pytest.raises(fem.FemError):
        batch.add_job(mid, ind, E0, NU0)
    batch.close()
