"""Parity of the HIP path against the FP64 CPU oracle (runs on an MI355X).

Every comparison runs the device kernels through the C ABI and the oracle on
the same seeded inputs. Tolerances:
  - FP64 path, single evaluations (gradient, energy, Hv): 1e-11 relative to
    the largest entry (summation order of ~24 element contributions per node);
  - FP32 path, single evaluations: 2e-5 relative to the largest entry
    (float rounding of O(10) operations per element contribution);
  - full solves: e_inf = max_i |u_i - u_i^ref| / max_i |u_i^ref| <= 1e-8 (FP64,
    both sides converged to 1e-10 relative residual) and <= 1e-4 (FP32 path,
    the stated accuracy target of the mixed-precision path).
"""
import numpy as np
import pytest

from paper_2103_16747_amd import fem, workload as W

pytestmark = pytest.mark.gpu

E0, NU0 = 0.3e6, 0.45


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def lib():
    return fem.load()


def e_inf(u, ref):
    return float(np.abs(u - ref).max() / max(np.abs(ref).max(), 1e-300))


def make_pair(oracle_lib, mesh, precision, ind=None, center=None):
    dev = fem.FemMesh(mesh.X, mesh.tets, mesh.fixed, precision=precision)
    dev.set_material(E0, NU0, 1100.0)
    orc = oracle_lib.Solver(mesh.X, mesh.tets, mesh.fixed, E=E0, nu=NU0)
    if ind is not None:
        c = ind.center(1) if center is None else center
        dev.set_indenter(ind.kind, ind.shape, ind.R, c, ind.k_penalty)
        orc.set_indenter(ind.kind, ind.shape, ind.R, c, ind.k_penalty)
    return dev, orc


MESHES = {
    "cube8": lambda: W.cube_block_mesh(),
    "tiny": lambda: W.block_mesh((1, 1, 1), (2e-3, 2e-3, 2e-3)),
    "fingertip5k": lambda: W.fingertip_mesh(5000),
    "fingertip50k": lambda: W.fingertip_mesh(50000),
}


@pytest.mark.parametrize("name", list(MESHES))
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_contact_eligible_nodes_match(oracle_lib, lib, name, precision):
    say("case", name, precision)
    mesh = MESHES[name]()
    dev, orc = make_pair(oracle_lib, mesh, precision)
    info = dev.info()
    assert info["n"] == mesh.n and info["m"] == mesh.m
    np.testing.assert_array_equal(info["eligible"], orc.eligible)
    assert info["n_eligible"] == int(orc.eligible.sum())


def indenter_for(mesh, kind, seed):
    """A seeded indenter pressed a little into the mesh's top region."""
    rng = np.random.default_rng(seed)
    top = mesh.X[:, 2].max()
    ctr = mesh.X[mesh.X[:, 2] >= top - 1e-12].mean(axis=0)
    shape = {W.SPHERE: [3e-3], W.CYLINDER: [1.5e-3, 2e-3], W.BOX: [1.2e-3, 1.0e-3, 0.8e-3],
             W.RING: [1.6e-3, 0.6e-3]}[kind]
    lead = {W.SPHERE: lambda: shape[0], W.CYLINDER: lambda: shape[1] / 2, W.BOX: lambda: shape[2],
            W.RING: lambda: shape[1]}[kind]()
    A = rng.normal(size=(3, 3)) * 0.15 + np.eye(3)
    Q, _ = np.linalg.qr(A)
    if np.linalg.det(Q) < 0:
        Q[:, 0] *= -1
    c = ctr + np.array([0.2e-3, -0.1e-3, lead - 0.3e-3])
    return W.Indentation(kind, np.array(shape), Q, c, np.array([0, 0, -1.0]), 0.0, 1)


@pytest.mark.parametrize("name", ["cube8", "fingertip5k", "fingertip50k"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("kind", [W.SPHERE, W.CYLINDER, W.BOX, W.RING])
def test_gradient_and_energy_parity(oracle_lib, lib, name, precision, kind):
    say("case", name, precision, kind)
    mesh = MESHES[name]()
    ind = indenter_for(mesh, kind, 100 + kind)
    dev, orc = make_pair(oracle_lib, mesh, precision, ind, center=ind.c0)
    u = W.random_displacement(mesh, 7 + kind, 0.01)
    dev.set_displacements(u)
    g, e, mj = dev.gradient()
    g_ref = orc.gradient(u)
    e_ref, mj_ref = orc.energy(u)
    tol = 1e-11 if precision == "fp64" else 2e-5
    scale = np.abs(g_ref).max()
    assert np.abs(g - g_ref).max() <= tol * scale
    assert e == pytest.approx(e_ref, rel=tol * 10)
    assert mj == pytest.approx(mj_ref, rel=tol * 10)
    ids, f, phi, Ft = dev.contact_patch()
    ids_r, f_r, phi_r, Ft_r = orc.contact_patch(u)
    if precision == "fp32":
        # u is rounded to float on upload; compare the patch computed by the
        # oracle at the rounded state (the device evaluates the contact law
        # in FP64 on both paths, so the bounds are the same).
        u32 = u.astype(np.float32).astype(np.float64)
        ids_r, f_r, phi_r, Ft_r = orc.contact_patch(u32)
    np.testing.assert_array_equal(ids, ids_r)
    fscale = max(np.abs(f_r).max(initial=0.0), 1e-30)
    np.testing.assert_allclose(f, f_r, rtol=1e-12, atol=1e-13 * fscale)
    np.testing.assert_allclose(phi, phi_r, rtol=1e-12, atol=1e-18)
    np.testing.assert_allclose(Ft, Ft_r, rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("name", ["cube8", "fingertip50k"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("contact_hessian", [0, 1])
def test_hessvec_parity(oracle_lib, lib, name, precision, contact_hessian):
    say("case", name, precision, contact_hessian)
    mesh = MESHES[name]()
    ind = indenter_for(mesh, W.SPHERE, 5)
    dev, orc = make_pair(oracle_lib, mesh, precision, ind, center=ind.c0)
    u = W.random_displacement(mesh, 11, 0.01)
    if precision == "fp32":
        u = u.astype(np.float32).astype(np.float64)
    dev.set_displacements(u)
    v = np.random.default_rng(3).normal(size=u.shape)
    if precision == "fp32":
        v = v.astype(np.float32).astype(np.float64)
    q = dev.hessvec(v, dev.default_params(contact_hessian=contact_hessian))
    q_ref = orc.hessvec(u, v, contact_full=contact_hessian)
    tol = 1e-11 if precision == "fp64" else 2e-5
    assert np.abs(q - q_ref).max() <= tol * np.abs(q_ref).max()


def tight(dev, precision):
    if precision == "fp64":
        return dev.default_params(newton_rtol=1e-10, cg_rtol=1e-10)
    return dev.default_params()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_cube_indentation_parity(oracle_lib, lib, precision):
    say("case cube indentation", precision)
    mesh = W.cube_block_mesh()
    ind = W.cube_sphere_indentation()
    dev, orc = make_pair(oracle_lib, mesh, precision)
    ref = orc.solve_indentation(ind, params=oracle_lib.default_params(newton_rtol=1e-11, cg_rtol=1e-11))
    worst = 0.0
    P = tight(dev, precision)
    for k in range(1, ind.steps + 1):
        dev.set_indenter(ind.kind, ind.shape, ind.R, ind.center(k), ind.k_penalty)
        info = dev.step(P)
        assert info["status"] >= 0, (k, info)   # FEM_OK or FEM_W_FLOOR; the bound below decides
        u = dev.displacements()
        worst = max(worst, e_inf(u, ref[k - 1][0]))
        say(k, info["newton_iters"], info["cg_iters"], "e_inf %.3e" % worst)
    bound = 1e-8 if precision == "fp64" else 1e-4
    assert worst <= bound
    ids, f, phi, Ft = dev.contact_patch()
    ids_r, f_r, phi_r, Ft_r = orc.contact_patch(ref[-1][0])
    np.testing.assert_array_equal(ids, ids_r)
    assert np.abs(Ft - Ft_r).max() <= (1e-7 if precision == "fp64" else 1e-3) * np.abs(Ft_r).max()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_fingertip_first_steps_parity(oracle_lib, lib, precision):
    """Full-size fingertip (50k tets), seeded indenter, first load steps taken
    at 10x the nominal increment."""
    mesh = W.fingertip_mesh(50000)
    for seed in (2001, 2003):
        say("case fingertip", precision, seed)
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
            assert err <= (1e-8 if precision == "fp64" else 1e-4)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_no_contact_step_is_immediate(lib, precision):
    mesh = W.cube_block_mesh()
    dev = fem.FemMesh(mesh.X, mesh.tets, mesh.fixed, precision=precision)
    dev.set_material(E0, NU0)
    dev.set_indenter(W.SPHERE, [1e-3], np.eye(3), [0.0, 0.0, 1.0])
    info = dev.step()
    assert info["status"] == 0 and info["newton_iters"] == 0 and info["g0_norm"] == 0.0
    assert np.all(dev.displacements() == 0.0)
    ids, f, phi, Ft = dev.contact_patch()
    assert len(ids) == 0 and np.all(Ft == 0)


def test_newton_cap_reports_not_converged_and_keeps_state(oracle_lib, lib):
    mesh = W.cube_block_mesh()
    ind = W.cube_sphere_indentation()
    dev, orc = make_pair(oracle_lib, mesh, "fp64", ind, center=ind.center(5))
    info = dev.step(dev.default_params(max_newton=1))
    assert info["status"] == fem.FEM_E_NOT_CONVERGED and info["newton_iters"] == 1
    u1 = dev.displacements()
    assert np.abs(u1).max() > 0
    # Continuing from the kept state converges.
    info = dev.step(dev.default_params(newton_rtol=1e-10, cg_rtol=1e-10))
    assert info["status"] >= 0
    ref, _ = orc.step(np.zeros((mesh.n, 3)), oracle_lib.default_params(newton_rtol=1e-11, cg_rtol=1e-11))
    assert e_inf(dev.displacements(), ref) <= 1e-8


def test_state_errors(lib):
    mesh = W.cube_block_mesh()
    dev = fem.FemMesh(mesh.X, mesh.tets, mesh.fixed)
    with pytest.raises(fem.FemError) as ei:
        dev.step()
    assert ei.value.code == fem.FEM_E_STATE
    with pytest.raises(fem.FemError):
        dev.set_material(-1.0, 0.3)
    with pytest.raises(fem.FemError):
        dev.set_indenter(W.SPHERE, [1e-3], 2 * np.eye(3), [0, 0, 0])
    bad = mesh.tets.copy()
    bad[7, [1, 2]] = bad[7, [2, 1]]
    with pytest.raises(fem.FemError) as ei:
        fem.FemMesh(mesh.X, bad, mesh.fixed)
    assert ei.value.code == fem.FEM_E_DEGENERATE
