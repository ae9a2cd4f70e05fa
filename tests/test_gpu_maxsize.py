"""The largest mesh of the workloads (the 120k-tet fingertip of the mixed-
resolution batch) against the FP64 oracle, and degenerate meshes (runs on an
MI355X). Tolerances as in the other parity tests: single evaluations 1e-11
(FP64) and 2e-5 (FP32) relative to the largest entry; solves e_inf <= 1e-8
(FP64, both sides converged to 1e-10 relative residual) and 1e-4 (FP32).
"""
import numpy as np
import pytest

from paper_2103_16747_amd import fem, workload as W
from test_gpu_parity import indenter_for

pytestmark = pytest.mark.gpu

E0, NU0 = 0.3e6, 0.45
SINGLE = {"fp64": 1e-11, "fp32": 2e-5}
SOLVE = {"fp64": 1e-8, "fp32": 1e-4}


def say(*a):
    print(*a, flush=True)


def e_inf(u, ref):
    return float(np.abs(u - ref).max() / max(np.abs(ref).max(), 1e-300))


@pytest.fixture(scope="module")
def tip120k():
    return W.fingertip_mesh(120000)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_fingertip120k_single_evaluations(oracle_lib, tip120k, precision):
    mesh = tip120k
    say("case 120k single evaluations", precision, mesh.m, "tets")
    ind = indenter_for(mesh, W.RING, 500)
    dev = fem.FemMesh(mesh.X, mesh.tets, mesh.fixed, precision=precision)
    dev.set_material(E0, NU0, 1100.0)
    dev.set_indenter(ind.kind, ind.shape, ind.R, ind.c0, ind.k_penalty)
    orc = oracle_lib.Solver(mesh.X, mesh.tets, mesh.fixed, E=E0, nu=NU0)
    orc.set_indenter(ind.kind, ind.shape, ind.R, ind.c0, ind.k_penalty)
    u = W.random_displacement(mesh, 51, 0.01)
    v = np.random.default_rng(52).normal(size=u.shape)
    if precision == "fp32":
        u = u.astype(np.float32).astype(np.float64)
        v = v.astype(np.float32).astype(np.float64)
    dev.set_displacements(u)
    g, e, mj = dev.gradient()
    g_ref = orc.gradient(u)
    e_ref, mj_ref = orc.energy(u)
    eg = np.abs(g - g_ref).max() / np.abs(g_ref).max()
    q = dev.hessvec(v, dev.default_params(contact_hessian=1))
    q_ref = orc.hessvec(u, v, contact_full=1)
    eq = np.abs(q - q_ref).max() / np.abs(q_ref).max()
    say("gradient e %.3e hessvec e %.3e energy e %.3e" % (eg, eq, abs(e - e_ref) / abs(e_ref)))
    assert eg <= SINGLE[precision] and eq <= SINGLE[precision]
    assert e == pytest.approx(e_ref, rel=10 * SINGLE[precision])
    assert mj == pytest.approx(mj_ref, rel=10 * SINGLE[precision])
    dev.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_fingertip120k_first_steps(oracle_lib, tip120k, precision):
    """A seeded job's first two load steps at ten times the nominal
    increment, through the single-mesh API."""
    mesh = tip120k
    ind = W.seat_on_mesh(W.random_indentation(2001, steps=10), mesh)
    say("case 120k first steps", precision, W.KIND_NAMES[ind.kind])
    orc = oracle_lib.Solver(mesh.X, mesh.tets, mesh.fixed, E=E0, nu=NU0)
    ref = orc.solve_indentation(ind, steps=2, params=oracle_lib.default_params(newton_rtol=1e-11, cg_rtol=1e-11))
    dev = fem.FemMesh(mesh.X, mesh.tets, mesh.fixed, precision=precision)
    dev.set_material(E0, NU0, 1100.0)
    P = dev.default_params(newton_rtol=1e-10, cg_rtol=1e-10) if precision == "fp64" else dev.default_params()
    for k in range(1, 3):
        dev.set_indenter(ind.kind, ind.shape, ind.R, ind.center(k), ind.k_penalty)
        info = dev.step(P)
        assert info["status"] >= 0, (k, info)
        err = e_inf(dev.displacements(), ref[k - 1][0])
        say(k, info["newton_iters"], info["cg_iters"], "e_inf %.3e" % err)
        assert err <= SOLVE[precision]
    dev.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_all_nodes_fixed_is_immediate(precision):
    """No free node: every step is immediate, displacements stay as
    prescribed and no contact force is reported on fixed nodes."""
    mesh = W.block_mesh((2, 2, 2), (2e-3, 2e-3, 2e-3))
    fixed = np.ones(mesh.n, dtype=np.uint8)
    dev = fem.FemMesh(mesh.X, mesh.tets, fixed, precision=precision)
    dev.set_material(E0, NU0, 1100.0)
    dev.set_indenter(W.SPHERE, [1e-3], np.eye(3), [1e-3, 1e-3, 2.5e-3])   # pressing into the block
    info = dev.step()
    assert info["status"] == 0 and info["newton_iters"] == 0
    assert np.all(dev.displacements() == 0.0)
    ids, f, phi, Ft = dev.contact_patch()
    assert len(ids) == 0 and np.all(Ft == 0.0)
    dev.close()
