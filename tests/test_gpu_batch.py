"""Batched indentation jobs on an MI355X: parity with the FP64 oracle, the same
result alone and in a mix of jobs (uneven meshes, different indenters), and
jobs joining a batch that is already running (continuous batching).

Tolerances: FP64 jobs against the oracle e_inf <= 1e-8 (both converged to a
1e-10 relative residual); FP32 jobs <= 1e-4. Alone vs in the mix: the two runs
execute the same kernels on the same state except for the order of LDS
atomic additions inside a tile, so they agree to the solve tolerance: 1e-9
(FP64) and 1e-5 (FP32) relative to max |u|.
"""
import numpy as np
import pytest

from paper_2103_16747_amd import fem, workload as W

pytestmark = pytest.mark.gpu
E0, NU0 = 0.3e6, 0.45


def say(*a):
    print(*a, flush=True)


def e_inf(u, ref):
    return float(np.abs(u - ref).max() / max(np.abs(ref).max(), 1e-300))


def tight(batch, precision):
    if precision == "fp64":
        return batch.default_params(newton_rtol=1e-10, cg_rtol=1e-10)
    return batch.default_params()


def cube_jobs():
    """The block-and-sphere schedule plus three other indenters on the block."""
    base = W.cube_sphere_indentation()
    jobs = [base]
    shapes = {W.CYLINDER: [1.5e-3, 2e-3], W.BOX: [1.5e-3, 1.2e-3, 1.0e-3], W.RING: [2.0e-3, 0.8e-3]}
    lead = {W.CYLINDER: 1e-3, W.BOX: 1.0e-3, W.RING: 0.8e-3}
    for kind in (W.CYLINDER, W.BOX, W.RING):
        c0 = np.array([5.2e-3, 4.9e-3, 10e-3 + lead[kind]])
        jobs.append(W.Indentation(kind, np.array(shapes[kind]), np.eye(3), c0, np.array([0.0, 0.0, -1.0]),
                                  0.8e-3, 8))
    return jobs


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_matches_oracle(oracle_lib, precision):
    mesh = W.cube_block_mesh()
    jobs = cube_jobs()
    batch = fem.FemBatch(len(jobs), precision)
    mid = batch.add_mesh(mesh.X, mesh.tets, mesh.fixed)
    ids = [batch.add_job(mid, j, E0, NU0) for j in jobs]
    say("batch", precision, "jobs", ids)
    assert batch.run(tight(batch, precision)) == 0
    orc = oracle_lib.Solver(mesh.X, mesh.tets, mesh.fixed, E=E0, nu=NU0)
    for jid, job in zip(ids, jobs):
        info = batch.job_info(jid)
        assert info["done"] == 1 and info["status"] == 0 and info["steps_ok"] == job.steps, info
        ref = orc.solve_indentation(job, params=oracle_lib.default_params(newton_rtol=1e-11, cg_rtol=1e-11))
        err = e_inf(batch.displacements(jid), ref[-1][0])
        say(W.KIND_NAMES[job.kind], "e_inf %.3e" % err, "newton", info["newton_iters"], "cg", info["cg_iters"])
        assert err <= (1e-8 if precision == "fp64" else 1e-4)
        ids_d, f, phi, Ft = batch.contact_patch(jid)
        ids_r, f_r, phi_r, Ft_r = orc.contact_patch(ref[-1][0])
        np.testing.assert_array_equal(ids_d, ids_r)
    batch.close()


def run_alone(mesh, job, precision, params_fn):
    b = fem.FemBatch(1, precision)
    mid = b.add_mesh(mesh.X, mesh.tets, mesh.fixed)
    jid = b.add_job(mid, job, E0, NU0)
    b.run(params_fn(b, precision))
    u = b.displacements(jid)
    b.close()
    return u


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_alone_equals_in_uneven_mix(precision):
    cube = W.cube_block_mesh()
    tip = W.fingertip_mesh(5000)
    tip_jobs = [W.seat_on_mesh(W.random_indentation(4000 + s, steps=6), tip) for s in range(3)]
    cjobs = cube_jobs()[:2]
    batch = fem.FemBatch(8, precision)
    m_cube = batch.add_mesh(cube.X, cube.tets, cube.fixed)
    m_tip = batch.add_mesh(tip.X, tip.tets, tip.fixed)
    mix = [(m_cube, cube, j) for j in cjobs] + [(m_tip, tip, j) for j in tip_jobs]
    ids = [batch.add_job(mid, j, E0, NU0) for mid, _, j in mix]
    batch.run(tight(batch, precision))
    tol = 1e-9 if precision == "fp64" else 1e-5
    for jid, (mid, mesh, job) in zip(ids, mix):
        info = batch.job_info(jid)
        assert info["done"] == 1 and info["steps_failed"] == 0, info
        alone = run_alone(mesh, job, precision, tight)
        err = e_inf(batch.displacements(jid), alone)
        say(precision, mesh.name, W.KIND_NAMES[job.kind], "alone vs mix %.3e" % err)
        assert err <= tol
    batch.close()


def test_job_joins_running_batch_and_slot_reuse():
    mesh = W.cube_block_mesh()
    jobs = cube_jobs()
    batch = fem.FemBatch(2, "fp64")
    mid = batch.add_mesh(mesh.X, mesh.tets, mesh.fixed)
    P = tight(batch, "fp64")
    a = batch.add_job(mid, jobs[0], E0, NU0)
    running = batch.run(P, max_rounds=3)
    assert running == 1
    assert batch.job_info(a)["done"] == 0
    b = batch.add_job(mid, jobs[1], E0, NU0)
    with pytest.raises(fem.FemError) as ei:
        batch.add_job(mid, jobs[2], E0, NU0)
    assert ei.value.code == fem.FEM_E_BUFFER
    assert batch.run(P) == 0
    for jid, job in ((a, jobs[0]), (b, jobs[1])):
        alone = run_alone(mesh, job, "fp64", tight)
        assert e_inf(batch.displacements(jid), alone) <= 1e-9
    batch.remove_job(a)
    c = batch.add_job(mid, jobs[2], E0, NU0)
    assert c == a
    assert batch.run(P) == 0
    alone = run_alone(mesh, jobs[2], "fp64", tight)
    assert e_inf(batch.displacements(c), alone) <= 1e-9
    batch.close()


def test_layout_covers_mesh():
    mesh = W.fingertip_mesh(50000)
    batch = fem.FemBatch(1, "fp32")
    mid = batch.add_mesh(mesh.X, mesh.tets, mesh.fixed)
    info = batch.mesh_info(mid)
    say(info)
    assert info["n_nodes"] == mesh.n and info["n_tets"] == mesh.m
    assert info["n_tiles"] >= mesh.m // 512
    assert mesh.n <= info["n_entries"] <= 2 * mesh.n
    batch.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_graph_replay_matches_stream_launches(precision):
    """Rounds replayed from captured graphs (many replays, with host state
    writes and synchronisations between them) give the results of rounds
    launched kernel by kernel; kernel timing records events for each of the
    three kernels."""
    mesh = W.cube_block_mesh()
    jobs = cube_jobs()
    out = {}
    for graphs in (1, 0):
        batch = fem.FemBatch(len(jobs), precision)
        batch.set_graphs(graphs)
        if not graphs:
            batch.set_kernel_timing(4)
        mid = batch.add_mesh(mesh.X, mesh.tets, mesh.fixed)
        ids = [batch.add_job(mid, j, E0, NU0) for j in jobs]
        assert batch.run(tight(batch, precision)) == 0
        out[graphs] = [batch.displacements(j) for j in ids]
        if not graphs:
            for k in (fem.FEM_KERNEL_TILE, fem.FEM_KERNEL_NODE, fem.FEM_KERNEL_FINALIZE):
                cnt, ms = batch.kernel_timing(k)
                launches = batch.kernel_launches(k)
                assert cnt > 0 and ms > 0 and launches >= cnt
        batch.close()
    tol = 1e-9 if precision == "fp64" else 1e-5
    for a, b in zip(out[1], out[0]):
        assert e_inf(a, b) <= tol


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_served_results_equal_alone(precision):
    """Staggered requests on two meshes through the serving loop: each result
    equals the same job solved alone, within the alone-vs-mix tolerance (1e-9
    FP64, 1e-5 FP32)."""
    from paper_2103_16747_amd.serve import IndentationServer, Request
    cube = W.cube_block_mesh()
    tip = W.fingertip_mesh(5000)
    jobs = cube_jobs()
    tip_jobs = [W.seat_on_mesh(W.random_indentation(4100 + s, steps=5), tip) for s in range(3)]
    reqs = [Request(i, 0.002 * i, "cube", j) for i, j in enumerate(jobs)]
    reqs += [Request(len(jobs) + i, 0.003 * i, "tip", j) for i, j in enumerate(tip_jobs)]
    batch = fem.FemBatch(5, precision)
    srv = IndentationServer(batch, {"cube": cube, "tip": tip}, hbm_budget=1 << 30, max_jobs=5,
                            params=tight(batch, precision), rounds_per_poll=2, keep_displacements=True)
    res = srv.serve(reqs, timeout=120)
    assert len(res) == len(reqs) and all(r.steps_failed == 0 for r in res)
    meshes = {"cube": cube, "tip": tip}
    for r in res:
        req = reqs[r.rid]
        alone = run_alone(meshes[req.mesh], req.indentation, precision, tight)
        err = e_inf(r.u, alone)
        say("served", precision, r.rid, req.mesh, "latency %.1f ms" % (r.latency * 1e3), "vs alone %.2e" % err)
        assert err <= (1e-9 if precision == "fp64" else 1e-5)
    batch.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_two_job_groups_match_one(precision):
    """Rounds split into two job groups on two streams (tile passes
    alternating between the groups) compute what one group computes: jobs on
    two meshes, run with one group, with two groups replayed from graphs, and
    with two groups launched kernel by kernel; the same bounds as alone vs
    in the mix."""
    meshes = [W.fingertip_mesh(5000), W.fingertip_mesh(50000)]
    jobs = []
    for i in range(10):
        mesh = meshes[i % 2]
        ind = W.seat_on_mesh(W.random_indentation(3000 + i), mesh)
        jobs.append((i % 2, W.Indentation(ind.kind, ind.shape, ind.R, ind.c0, ind.direction, ind.depth / 10, 10,
                                          ind.k_penalty, seed=3000 + i)))
    runs = {}
    for name, groups, graphs in (("one group", 1, 1), ("two groups", 2, 1), ("two groups, no graphs", 2, 0)):
        b = fem.FemBatch(len(jobs), precision)
        b.set_option(fem.FEM_OPT_GROUPS, groups)
        b.set_graphs(graphs)
        mids = [b.add_mesh(m.X, m.tets, m.fixed) for m in meshes]
        ids = [b.add_job(mids[k], job, E0, NU0) for k, job in jobs]
        say("case", precision, name)
        assert b.run(tight(b, precision)) == 0
        runs[name] = [b.displacements(j) for j in ids]
        for j in ids:
            info = b.job_info(j)
            assert info["done"] == 1 and info["steps_ok"] + info["steps_failed"] == 10, info
        b.close()
    bound = 1e-9 if precision == "fp64" else 1e-5
    for name in ("two groups", "two groups, no graphs"):
        errs = [e_inf(u, ref) for u, ref in zip(runs[name], runs["one group"])]
        say(precision, name, "vs one group: max e_inf %.3e" % max(errs))
        assert max(errs) <= bound, errs


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_deterministic_mode_is_bitwise(precision):
    """The fixed-order tile sums (FEM_OPT_DETERMINISTIC): each job's result is
    bitwise the same alone, in a mix of meshes, laws and indenters replayed
    from graphs, and in the same mix split into two job groups launched
    kernel by kernel; and the default mode (LDS atomics, whose sums follow
    the order of wavefronts) agrees with it within the alone-vs-mix bounds."""
    cube = W.cube_block_mesh()
    tip = W.fingertip_mesh(5000)
    mix = [(cube, j, E0, NU0) for j in cube_jobs()[:2]]
    for s, model in ((4200, 0), (4201, 1), (4202, 0)):
        base = W.seat_on_mesh(W.random_indentation(s, steps=6), tip)
        ind = W.Indentation(base.kind, base.shape, base.R, base.c0, base.direction, base.depth * 0.6, 6,
                            base.k_penalty, seed=s, model=model, friction=0.3 if model else 0.0,
                            friction_eps=1e-5)
        mix.append((tip, ind, 1.55e6 if model else E0, 0.316 if model else NU0))

    def run(jobs, det, groups=1, graphs=1):
        b = fem.FemBatch(len(jobs), precision)
        b.set_option(fem.FEM_OPT_DETERMINISTIC, det)
        b.set_option(fem.FEM_OPT_GROUPS, groups)
        b.set_graphs(graphs)
        mids = {}
        ids = []
        for mesh, ind, E, nu in jobs:
            if mesh.name not in mids:
                mids[mesh.name] = b.add_mesh(mesh.X, mesh.tets, mesh.fixed)
            ids.append(b.add_job(mids[mesh.name], ind, E, nu))
        assert b.run(tight(b, precision)) == 0
        for j, (_, ind, _, _) in zip(ids, jobs):
            info = b.job_info(j)
            assert info["done"] == 1 and info["steps_ok"] + info["steps_failed"] == ind.steps, info
        out = [b.displacements(j) for j in ids]
        b.close()
        return out

    say("case", precision, "deterministic, mix")
    det_mix = run(mix, 1)
    say("case", precision, "deterministic, two groups, no graphs")
    det_groups = run(mix, 1, groups=2, graphs=0)
    say("case", precision, "default mode, mix")
    atomic_mix = run(mix, 0)
    bound = 1e-9 if precision == "fp64" else 1e-5
    for i, job in enumerate(mix):
        say("case", precision, "deterministic, alone", i)
        alone = run([job], 1)[0]
        np.testing.assert_array_equal(det_mix[i], alone)
        np.testing.assert_array_equal(det_groups[i], alone)
        err = e_inf(atomic_mix[i], alone)
        say(precision, job[0].name, W.KIND_NAMES[job[1].kind], "model", job[1].model,
            "default vs deterministic %.3e" % err)
        assert err <= bound
