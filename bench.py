#!/usr/bin/env python3
"""Benchmark of batched indentation solves on one MI355X.

A step is one batch: 256 independent indentation jobs on the synthetic
50k-tet fingertip, each with its own seeded rigid indenter (sphere, cylinder,
box or ring; random surface point, tilt up to 30 degrees and depth up to
3 mm), pressed in over 100 quasi-static load steps and solved to the end.
All jobs run concurrently through one launch sequence (FP32 element math and
CG vectors, FP64 reductions); the mesh and every job's state are resident in
HBM before the timed region.

Printed as one JSON line: solves/s and tet-updates/s of the batched FP32
path; per-job completion latency p50/p99 within the batch; the same batch on
the FP64 path; the plain FP64 single-instance path (one job at a time) for
comparison; the roofline of the dominant kernel, event-timed on the library's
stream during the timed region; and the FP64 CPU oracle timed on a bounded
sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0
METRIC = "FEM indentation solves/s + tet-updates/s, FP32 vs FP64 path; p50/p99 latency"


# Algorithmic arithmetic per tet of the two tile-kernel paths (an FMA counts
# two; one transcendental counts one; FP64 LDS accumulation and conversions
# are not counted):
#   Hessian-vector: G from u (54), J - 1 (30), ln J series and c (16),
#   F^-T (40), dG from p (54), A = F^-1 dG and its trace (47), dP (91),
#   nodal forces (60), p.q (25)                                  -> 417
#   element: G (54), J - 1 (30), ln J (1), energy and magnitude (36),
#   F^-T (40), P (82), nodal forces (60), node diagonal blocks (161) -> 464
FLOPS_PER_TET = {"hv": 417, "element": 464}
# The co-rotational law (same counting): both passes share G, J - 1, dG or
# the node blocks, nodal forces and p.q with the Neo-Hookean ones (223 for
# the Hessian-vector pass, 305 for the element pass). Per tet the law adds
# the polar rotation, 3 + 83 per Newton iteration; the Hessian-vector pass
# then forms E = sym(R^T F) - I (102), R^T dG, the rotation rate w and dP
# (184); the element pass forms E = (C - I)(S + I)^-1 without cancellation
# (243), tr E, |E|^2, the energy and P = R (2 mu E + lam tr E I) (81). The
# iteration count is data-dependent: 2.2 per tet on average over the
# co-rotational fingertip states at 20-100 % of the indentation depth, which
# gives 695 and 815.
POLAR_ITERS = 2.2
FLOPS_PER_TET_CR = {"hv": round(223 + 3 + 83 * POLAR_ITERS + 102 + 184),
                    "element": round(305 + 3 + 83 * POLAR_ITERS + 243 + 81)}
FP32_VECTOR_PEAK_TFLOPS = 157.3      # 256 CU x 64 lanes x 2 x 2.4 GHz x 2 (packed FP32)
FP32_NONPACKED_PEAK_TFLOPS = 78.6    # the same without packed FP32, which the library is compiled without


def tile_bytes(info, word, hv_passes, el_passes, launches):
    """Algorithmic HBM bytes per launch of the tile kernel, averaged over
    `launches` launches that made hv_passes Hessian-vector passes and
    el_passes element passes in all (ideal reuse: every value read or written
    once per pass; the mesh constants once per launch).

    Shared per launch: packed local ids (4 B/tet), D_m^-1 and V (10 words per
    tet), the entry -> node map (4 B per entry).
    Hessian-vector pass, per job: reads of u, z, p_prev (9 words per node),
    write of the q partials (3 words per entry), contact blocks (6 words per
    eligible node).
    Element pass, per job: reads of u and dx (6 words per node), write of the
    gradient + block partials (9 words per entry), contact node coordinates
    (3 doubles) and contact outputs (9 words) per eligible node.
    """
    n, m, nent, nc = info["n_nodes"], info["n_tets"], info["n_entries"], info["n_eligible"]
    shared = m * (4 + 10 * word) + 4 * nent
    hv = 9 * word * n + 3 * word * nent + 6 * word * nc
    el = 6 * word * n + 9 * word * nent + (24 + 9 * word) * nc
    return shared + (hv_passes * hv + el_passes * el) / max(launches, 1)


def progress(*a):
    print(*a, file=sys.stderr, flush=True)


def run_batched(mesh, inds, precision, timed_steps, warm_steps, timing_every=0, track_latency=True,
                material=(0.3e6, 0.45)):
    from paper_2103_16747_amd import fem

    batch = fem.FemBatch(len(inds), precision)
    mid = batch.add_mesh(mesh.X, mesh.tets, mesh.fixed)
    info = batch.mesh_info(mid)
    jobs = [batch.add_job(mid, ind, *material) for ind in inds]
    P = batch.default_params()
    for _ in range(warm_steps):
        for j, ind in zip(jobs, inds):
            batch.restart_job(j, ind, *material)
        batch.run(P)
        progress(f"warm-up batch {precision} done")
    if timing_every:
        batch.set_kernel_timing(timing_every)
    walls, lat, tu, failed, floor, hv, gp = [], [], 0, 0, 0, 0, 0
    for _ in range(timed_steps):
        for j, ind in zip(jobs, inds):
            batch.restart_job(j, ind, *material)
        t0 = time.perf_counter()
        done_at = {}
        running = len(jobs)
        pending = list(jobs)
        while running:
            prev = running
            running = batch.run(P, max_rounds=8 if track_latency else 0)
            now = time.perf_counter() - t0
            # completions are looked up only when the running count fell
            if track_latency and running < prev:
                for j in pending:
                    if batch.job_info(j)["done"]:
                        done_at[j] = now
                pending = [j for j in pending if j not in done_at]
        walls.append(time.perf_counter() - t0)
        progress(f"batched {precision}: {len(jobs)} jobs in {walls[-1]:.2f} s")
        infos = [batch.job_info(j) for j in jobs]
        tu += sum(i["tet_updates"] for i in infos)
        failed += sum(i["steps_failed"] for i in infos)
        floor += sum(i["steps_floor"] for i in infos)
        hv += sum(i["hv_products"] for i in infos)
        gp += sum(i["grad_passes"] for i in infos)
        lat += list(done_at.values())
    timing = None
    if timing_every:
        timing = {k: batch.kernel_timing(k) + (batch.kernel_launches(k),)
                  for k in (fem.FEM_KERNEL_TILE, fem.FEM_KERNEL_NODE, fem.FEM_KERNEL_FINALIZE)}
        batch.set_kernel_timing(0)
    finals = [batch.displacements(j) for j in jobs[:4]]
    stats = [batch.job_info(j) for j in jobs]
    # data-generation outputs of the finished jobs: per-tet stress and
    # displacement statistics (device kernels; the stress copy to the host
    # is included)
    t0 = time.perf_counter()
    nout = min(len(jobs), 32)
    for j in jobs[:nout]:
        batch.tet_stress(j)
        batch.displacement_stats(j)
    out_ms = (time.perf_counter() - t0) / nout * 1e3
    batch.close()
    return {"walls": walls, "lat": lat, "tet_updates": tu, "failed_steps": failed, "floor_steps": floor,
            "outputs_ms_per_job": out_ms,
            "timing": timing, "hv_passes": hv, "grad_passes": gp, "layout": info, "finals": finals, "stats": stats}


def run_single(mesh, inds, precision):
    """One job at a time through the single-mesh API (create once, then
    100 fem_step calls per job)."""
    from paper_2103_16747_amd import fem

    dev = fem.FemMesh(mesh.X, mesh.tets, mesh.fixed, precision=precision)
    dev.set_material(0.3e6, 0.45, 1100.0)
    zeros = np.zeros((mesh.n, 3))
    walls, tu, failed = [], 0, 0
    for ind in inds:
        t0 = time.perf_counter()
        dev.set_displacements(zeros)
        for k in range(1, ind.steps + 1):
            dev.set_indenter(ind.kind, ind.shape, ind.R, ind.center(k), ind.k_penalty)
            info = dev.step()
            tu += info["tet_updates"]
            failed += info["status"] != 0
        walls.append(time.perf_counter() - t0)
        progress(f"single {precision}: job {ind.seed} in {walls[-1]:.2f} s")
    dev.close()
    return {"walls": walls, "tet_updates": tu, "failed_steps": failed}


def cpu_baseline(mesh, ind, seconds):
    import oracle

    orc = oracle.Solver(mesh.X, mesh.tets, mesh.fixed, E=0.3e6, nu=0.45)
    u = np.zeros((mesh.n, 3))
    t0 = time.perf_counter()
    steps, passes = 0, 0
    for k in range(1, ind.steps + 1):
        orc.set_indenter(ind.kind, ind.shape, ind.R, ind.center(k), ind.k_penalty)
        u, info = orc.step(u)
        steps += 1
        passes += info["grad_passes"] + info["energy_passes"] + info["hv_products"]
        if time.perf_counter() - t0 >= seconds:
            break
        if steps % 10 == 0:
            progress(f"cpu oracle: {steps} load steps")
    el = time.perf_counter() - t0
    return {"value": (steps / ind.steps) / el, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "tet_updates_per_s": mesh.m * passes / el,
            "sample": f"FP64 oracle, one thread, the first {steps} of {ind.steps} load steps of job seed {ind.seed} "
                      f"on the {mesh.m}-tet fingertip ({el:.1f} s); solves/s = ({steps}/{ind.steps}) / time"}


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_tile_fingertip50k_traffic.json")


def measured_traffic():
    """HBM bytes per tile-kernel launch from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE runs (copy-calibrated), or None when they are
    missing or were taken on a different kernel source."""
    from paper_2103_16747_amd.profiling import kernel_source_hash

    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as f:
        t = json.load(f)
    if t.get("kernel_source_sha256") != kernel_source_hash():
        return None
    return t["traffic_bytes_per_dispatch"]


FP64_VECTOR_PEAK_TFLOPS = 78.6      # 256 CU x 64 lanes x 2 x 2.4 GHz (FP64 vector)


def roofline(r, word, flops_per_tet=FLOPS_PER_TET, kname=None, peak=FP32_VECTOR_PEAK_TFLOPS):
    """Roofline of the tile kernel (the dominant one) over the timed region:
    algorithmic flops per launch (the passes the jobs made, times the tets per
    pass and FLOPS_PER_TET, over the number of launches) divided by the mean
    event-timed duration of the sampled launches."""
    from paper_2103_16747_amd import fem

    tm = r["timing"]
    if not tm:
        return None, None
    per = {}
    for name, k in (("tile", fem.FEM_KERNEL_TILE), ("node", fem.FEM_KERNEL_NODE), ("finalize", fem.FEM_KERNEL_FINALIZE)):
        cnt, ms, launches = tm[k]
        per[name] = {"sampled": cnt, "launches": launches, "avg_us": (ms / cnt * 1e3) if cnt else None}
    t = per["tile"]
    if not t["sampled"]:
        return None, None
    m = r["layout"]["n_tets"]
    flops = m * (r["hv_passes"] * flops_per_tet["hv"] + r["grad_passes"] * flops_per_tet["element"])
    per_launch = flops / t["launches"]
    avg_s = t["avg_us"] * 1e-6
    achieved = per_launch / avg_s / 1e12
    byts = tile_bytes(r["layout"], word, r["hv_passes"], r["grad_passes"], t["launches"])
    if kname is None:
        kname = "k_tile<float, LAW_NH>" if word == 4 else "k_tile<double, LAW_NH>"
    out = {"bound": "alu", "kernel": kname, "achieved": achieved, "peak": peak,
           "unit": "TFLOP/s", "frac": achieved / peak, "traffic": measured_traffic() if word == 4 else None}
    if word == 4:
        out["frac_of_non_packed_peak"] = achieved / FP32_NONPACKED_PEAK_TFLOPS
    out.update({"avg_launch_us": t["avg_us"], "sampled_launches": t["sampled"], "launches": t["launches"],
                "flops_per_launch": per_launch,
                "tet_updates_per_launch": m * (r["hv_passes"] + r["grad_passes"]) / t["launches"],
                "hbm_model": {"algorithmic_bytes_per_launch": byts, "GB_per_s": byts / avg_s / 1e9,
                              "frac_of_hbm_peak": byts / avg_s / 1e9 / HBM_PEAK_GBS}})
    return out, {k: v["avg_us"] for k, v in per.items()}


RESOLUTIONS = (5000, 20000, 50000, 120000)


def uneven_jobs(count, seed0):
    """Seeded mix: each job's resolution uniform over RESOLUTIONS, then its
    indenter from the job seed."""
    from paper_2103_16747_amd import workload as W

    meshes = {r: W.fingertip_mesh(r) for r in RESOLUTIONS}
    rng = W.Xoshiro256ss(seed0)
    jobs = []
    for i in range(count):
        res = RESOLUTIONS[rng.below(len(RESOLUTIONS))]
        jobs.append((res, W.seat_on_mesh(W.random_indentation(seed0 + 1 + i), meshes[res])))
    return meshes, jobs


def bench_uneven(args):
    """64 jobs at mixed resolution in one batch, shapes from the autotuner,
    against the same jobs solved one at a time (FP32 path both)."""
    from paper_2103_16747_amd import autotune, fem

    meshes, jobs = uneven_jobs(64, 4000)
    tuned = autotune.tune([meshes[r] for r in RESOLUTIONS], "fp32", log=progress)
    progress(f"autotune: tile {tuned['tile_tets']} chunk {tuned['chunk']}")
    batch = fem.FemBatch(len(jobs), "fp32")
    batch.set_option(fem.FEM_OPT_TILE_TETS, tuned["tile_tets"])
    batch.set_option(fem.FEM_OPT_ROUND_STEPS, tuned["chunk"])
    mids = {r: batch.add_mesh(meshes[r].X, meshes[r].tets, meshes[r].fixed) for r in RESOLUTIONS}
    ids = [batch.add_job(mids[r], ind) for r, ind in jobs]
    batch.run()
    for j, (r, ind) in zip(ids, jobs):
        batch.restart_job(j, ind)
    t0 = time.perf_counter()
    batch.run()
    wall = time.perf_counter() - t0
    infos = [batch.job_info(j) for j in ids]
    batch.close()
    progress(f"uneven batch: {len(jobs)} jobs in {wall:.2f} s")
    # unbatched reference: the first job of each resolution, one at a time
    solo = {}
    for r in RESOLUTIONS:
        ind = next(ind for rr, ind in jobs if rr == r)
        single = run_single(meshes[r], [ind], "fp32")
        solo[r] = single["walls"][0]
    per_job_solo = sum(solo[r] for r, _ in jobs)
    tu = sum(i["tet_updates"] for i in infos)
    return {"metric": METRIC, "value": len(jobs) / wall, "unit": "solves/s", "n_gpus": 1, "steps": 1,
            "warmup": 1, "ms_per_step": wall * 1e3, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "uneven batch: 64 synthetic-fingertip jobs at 5k/20k/50k/120k tets (uniform mix), "
                                   "seeded indenters, 100 load steps each",
                       "mix": {str(r): sum(1 for rr, _ in jobs if rr == r) for r in RESOLUTIONS},
                       "autotuned": {"tile_tets": tuned["tile_tets"], "chunk": tuned["chunk"]}},
            "tet_updates_per_s": tu / wall, "failed_load_steps": sum(i["steps_failed"] for i in infos),
            "unbatched_estimate": {"solves_per_s": len(jobs) / per_job_solo,
                                   "per_resolution_s": {str(r): solo[r] for r in RESOLUTIONS},
                                   "note": "one job per resolution timed alone; the batch's jobs summed at those times"},
            "speedup_vs_unbatched": per_job_solo / wall,
            "autotune_table": tuned["table"]}


def bench_serving(args):
    """Poisson streams of mixed-resolution jobs through the serving loop
    (admission by HBM footprint, continuous batching); p50/p99 latency and
    solves/s per arrival rate, against one-at-a-time FP64 solves."""
    from paper_2103_16747_amd import fem, workload as W
    from paper_2103_16747_amd.serve import IndentationServer, Request, latency_summary

    meshes, jobs = uneven_jobs(args.requests, 5000)
    keyed = {str(r): meshes[r] for r in RESOLUTIONS}
    out = {"metric": METRIC, "unit": "ms", "n_gpus": 1, "higher_is_better": False, "data": "synthetic",
           "dtype": "f32", "config": {"workload": f"serving: Poisson arrivals of {args.requests} mixed-resolution "
                                                  "fingertip jobs per rate, 100 load steps each",
                                      "hbm_budget_GiB": 64}, "rates": {}}
    for rate in [float(x) for x in args.rates.split(",")]:
        arrivals = W.poisson_arrivals(int(rate * 1000), rate, len(jobs))
        reqs = [Request(i, float(t), str(r), ind) for i, (t, (r, ind)) in enumerate(zip(arrivals, jobs))]
        batch = fem.FemBatch(len(jobs), "fp32")
        srv = IndentationServer(batch, keyed, hbm_budget=64 << 30, max_jobs=len(jobs), rounds_per_poll=2)
        res = srv.serve(reqs, timeout=600)
        summ = latency_summary(res)
        summ["peak_running"] = srv.stats.peak_running
        out["rates"][str(rate)] = summ
        batch.close()
        progress(f"serving rate {rate}: p50 {summ['p50_ms']:.0f} ms p99 {summ['p99_ms']:.0f} ms "
                 f"{summ['solves_per_s']:.1f} solves/s")
    # one-at-a-time FP64 reference on the first job of each resolution
    ref = {}
    for r in RESOLUTIONS:
        ind = next(ind for rr, ind in jobs if rr == r)
        ref[str(r)] = run_single(meshes[r], [ind], "fp64")["walls"][0]
    mean_one = sum(ref[str(r)] for r, _ in jobs) / len(jobs)
    out["fp64_one_at_a_time"] = {"solves_per_s": 1.0 / mean_one, "per_resolution_s": ref}
    last = out["rates"][max(out["rates"], key=float)]
    out["value"] = last["p99_ms"]
    return out


def bench_dynamic(args):
    """The batched workload as implicit time steps: 256 fingertip jobs, each
    step a backward-Euler step of dt = 1e-4 s (the paper's time step) with
    lumped masses at 1100 kg/m^3, the indenter moving depth/100 per step.
    The first jobs' first steps are checked against stored FP64 oracle
    results (tests/golden/fingertip50k_dynamic_oracle.npz)."""
    from paper_2103_16747_amd import fem, workload as W

    mesh = W.fingertip_mesh(50000)
    dt, rho = 1e-4, 1100.0
    inds = []
    for i in range(args.jobs):
        ind = W.seat_on_mesh(W.random_indentation(3000 + i), mesh)
        ind.dt, ind.density = dt, rho
        inds.append(ind)
    batch = fem.FemBatch(len(inds), "fp32")
    mid = batch.add_mesh(mesh.X, mesh.tets, mesh.fixed)
    info = batch.mesh_info(mid)
    jobs = [batch.add_job(mid, ind) for ind in inds]
    batch.run()
    progress("warm-up dynamic batch done")
    walls, tu, failed, lat = [], 0, 0, []
    for _ in range(args.steps):
        for j, ind in zip(jobs, inds):
            batch.restart_job(j, ind)
        t0 = time.perf_counter()
        done_at, running = {}, len(jobs)
        pending = list(jobs)
        while running:
            prev = running
            running = batch.run(max_rounds=8)
            now = time.perf_counter() - t0
            if running < prev:
                for j in pending:
                    if batch.job_info(j)["done"]:
                        done_at[j] = now
                pending = [j for j in pending if j not in done_at]
        walls.append(time.perf_counter() - t0)
        progress(f"dynamic batch: {len(jobs)} jobs in {walls[-1]:.2f} s")
        infos = [batch.job_info(j) for j in jobs]
        tu += sum(i["tet_updates"] for i in infos)
        failed += sum(i["steps_failed"] for i in infos)
        lat += list(done_at.values())
    stats = [batch.job_info(j) for j in jobs]
    batch.close()
    # the first jobs' first time steps against stored FP64 oracle results
    errs = {}
    gold_path = os.path.join(ROOT, "tests", "golden", "fingertip50k_dynamic_oracle.npz")
    if os.path.exists(gold_path):
        gold = np.load(gold_path)
        k_check = int(gold["steps"])
        for seed in (int(x) for x in gold["seeds"]):
            ind = inds[seed - 3000]
            short = W.Indentation(ind.kind, ind.shape, ind.R, ind.c0, ind.direction, ind.depth * k_check / ind.steps,
                                  k_check, ind.k_penalty, dt=dt, density=rho)
            b1 = fem.FemBatch(1, "fp32")
            j1 = b1.add_job(b1.add_mesh(mesh.X, mesh.tets, mesh.fixed), short)
            b1.run()
            u_ref, v_ref = gold[f"u_{seed}"], gold[f"v_{seed}"]
            errs[str(seed)] = {"steps": k_check,
                               "u": float(np.abs(b1.displacements(j1) - u_ref).max() / np.abs(u_ref).max()),
                               "v": float(np.abs(b1.velocities(j1) - v_ref).max() / np.abs(v_ref).max())}
            b1.close()
    wall = sum(walls)
    lat_ms = np.array(lat) * 1e3
    K, J = args.steps, len(jobs)
    return {"metric": METRIC, "value": K * J / wall, "unit": "solves/s", "n_gpus": 1, "steps": K, "warmup": 1,
            "ms_per_step": wall / K * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32", "data": "synthetic",
            "config": {"workload": f"implicit dynamics: {J} jobs on the synthetic 50k-tet fingertip, seeded indenters, "
                                   "100 backward-Euler steps of 1e-4 s each (lumped mass, 1100 kg/m^3)",
                       "mesh_tets": mesh.m, "tiles": info["n_tiles"]},
            "tet_updates_per_s": tu / wall, "failed_load_steps": failed,
            "latency_ms": {"p50": float(np.percentile(lat_ms, 50)), "p99": float(np.percentile(lat_ms, 99))},
            "cg_iters_per_job": float(np.mean([s["cg_iters"] for s in stats])),
            "newton_iters_per_job": float(np.mean([s["newton_iters"] for s in stats])),
            "e_inf_vs_fp64_oracle_first_steps": errs}


VARIANTS = {
    # name: (law, E, nu, depth factor, friction, dt, description)
    "corotational": (1, 1.55e6, 0.316, 0.5, 0.0, 0.0,
                     "co-rotational batched indentation: {J} jobs on the synthetic 50k-tet fingertip, E = 1.55 MPa, "
                     "nu = 0.316, seeded indenters at half depth (up to 1.5 mm), 100 quasi-static load steps each"),
    "friction": (0, 0.3e6, 0.45, 1.0, 0.783, 0.0,
                 "batched indentation with Coulomb friction 0.783 (lagged, smoothed over 10 um): {J} jobs on the "
                 "synthetic 50k-tet fingertip, seeded indenters, 100 quasi-static load steps each"),
    "simulator": (1, 1.55e6, 0.316, 0.5, 0.783, 1e-4,
                  "the paper's simulator model: co-rotational skin (E = 1.55 MPa, nu = 0.316), Coulomb friction "
                  "0.783, backward-Euler steps of 1e-4 s (1100 kg/m^3); {J} jobs on the synthetic 50k-tet "
                  "fingertip, seeded indenters at half depth, 100 steps each"),
}


def bench_variant(args, name):
    """The batched workload (256 jobs on the 50k fingertip, FP32 path) with
    the co-rotational law of the paper's own simulator (E = 1.55 MPa,
    nu = 0.316, Sec. III-A), with Coulomb friction (coefficient 0.783), or
    with both and implicit time steps of 1e-4 s, and the roofline of the
    tile kernel instance that runs. Co-rotational variants halve the
    indentation depths (up to 1.5 mm): the law has no barrier against
    inversion, and boxes and rings pressed through most of the 3 mm skin
    invert elements (the oracle fails the same load steps)."""
    from paper_2103_16747_amd import workload as W

    law, E, nu, depth_f, mu_f, dt, desc = VARIANTS[name]
    mesh = W.fingertip_mesh(50000)
    inds = []
    for i in range(args.jobs):
        ind = W.seat_on_mesh(W.random_indentation(3000 + i), mesh)
        ind.model = law
        ind.depth *= depth_f
        ind.friction, ind.friction_eps = mu_f, 1e-5
        ind.dt, ind.density = dt, 1100.0
        inds.append(ind)
    r = run_batched(mesh, inds, "fp32", args.steps, args.warmup, args.timing_every, material=(E, nu))
    K, J = args.steps, args.jobs
    wall = sum(r["walls"])
    lat_ms = np.array(r["lat"]) * 1e3
    out = {"metric": METRIC, "value": K * J / wall, "unit": "solves/s", "n_gpus": 1, "steps": K,
           "warmup": args.warmup, "ms_per_step": wall / K * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": desc.format(J=J), "jobs_per_step": J, "mesh_tets": mesh.m},
           "tet_updates_per_s": r["tet_updates"] / wall,
           "latency_ms": {"p50": float(np.percentile(lat_ms, 50)), "p99": float(np.percentile(lat_ms, 99))},
           "failed_load_steps": r["failed_steps"], "floor_load_steps": r["floor_steps"],
           "cg_iters_per_job": float(np.mean([s["cg_iters"] for s in r["stats"]])),
           "newton_iters_per_job": float(np.mean([s["newton_iters"] for s in r["stats"]]))}
    fpt = FLOPS_PER_TET_CR if law == 1 else FLOPS_PER_TET
    out["flops_per_tet"] = fpt
    if law == 1:
        out["polar_iterations_assumed"] = POLAR_ITERS
    rl, kav = roofline(r, 4, fpt, "k_tile<float, LAW_CR>" if law == 1 else "k_tile<float, LAW_NH>")
    if rl:
        rl["traffic"] = None      # counters are taken on the default workload only
        out["roofline"] = rl
        out["kernel_avg_us"] = kav
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2, help="timed batches")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--jobs", type=int, default=256)
    ap.add_argument("--single-jobs", type=int, default=3, help="jobs timed one at a time on the FP64 path")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-single", action="store_true")
    ap.add_argument("--timing-every", type=int, default=8)
    ap.add_argument("--config", choices=("batched", "uneven", "serving", "dynamic", "corotational", "friction",
                                         "simulator"),
                    default="batched",
                    help="batched: 256 jobs on the 50k fingertip (default); uneven: 64 jobs at 5k-120k tets with "
                         "autotuned shapes; serving: Poisson request streams through the serving loop; dynamic: "
                         "the batched workload as implicit time steps of 1e-4 s; corotational: the batched workload under the "
                         "co-rotational law; friction: with Coulomb friction 0.783; simulator: co-rotational, "
                         "friction and implicit steps together")
    ap.add_argument("--rates", default="10,50,200,500", help="serving: arrival rates (req/s)")
    ap.add_argument("--requests", type=int, default=160, help="serving: requests per rate")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="before the solves, one device copy of this many MiB (calibrates rocprofv3 byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: each batch of indentation jobs runs on a single MI355X and the "
              "library has no multi-GPU path; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2103_16747_amd import fem, workload as W

    assert torch.cuda.is_available(), "no GPU visible"
    fem.load()
    if args.copy_mb > 0:
        src = torch.ones(args.copy_mb << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.config == "uneven":
        print(json.dumps(bench_uneven(args)), flush=True)
        return
    if args.config == "serving":
        print(json.dumps(bench_serving(args)), flush=True)
        return
    if args.config == "dynamic":
        print(json.dumps(bench_dynamic(args)), flush=True)
        return
    if args.config in VARIANTS:
        print(json.dumps(bench_variant(args, args.config)), flush=True)
        return
    mesh = W.fingertip_mesh(50000)
    inds = [W.seat_on_mesh(W.random_indentation(3000 + i), mesh) for i in range(args.jobs)]

    torch.cuda.synchronize()
    r32 = run_batched(mesh, inds, "fp32", args.steps, args.warmup, args.timing_every)
    torch.cuda.synchronize()
    K, J = args.steps, args.jobs
    wall = sum(r32["walls"])
    lat_ms = np.array(r32["lat"]) * 1e3
    out = {
        "metric": METRIC,
        "value": K * J / wall,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": wall / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"batched indentation: {J} jobs on the synthetic 50k-tet fingertip, seeded indenters "
                        f"(seeds 3000..{3000 + J - 1}), 100 quasi-static load steps each, all jobs concurrent",
            "jobs_per_step": J, "mesh_tets": mesh.m, "mesh_nodes": mesh.n,
            "tiles": r32["layout"]["n_tiles"], "tile_entries": r32["layout"]["n_entries"],
            "contact_eligible_nodes": r32["layout"]["n_eligible"],
            "precision": "fp32 element math and CG vectors; fp64 dots, norms, energies, Newton test, contact",
            "solver": "Newton + block-Jacobi PCG (matrix-free), Armijo line search, exact contact Hessian",
        },
        "tet_updates_per_s": r32["tet_updates"] / wall,
        "latency_ms": {"p50": float(np.percentile(lat_ms, 50)), "p99": float(np.percentile(lat_ms, 99)),
                       "mode": "job completion time from batch start, all jobs submitted together"},
        "failed_load_steps": r32["failed_steps"],
        "floor_load_steps": r32["floor_steps"],
        "cg_iters_per_job": float(np.mean([s["cg_iters"] for s in r32["stats"]])),
        "outputs_ms_per_job": r32["outputs_ms_per_job"],
        "newton_iters_per_job": float(np.mean([s["newton_iters"] for s in r32["stats"]])),
    }
    gold_path = os.path.join(ROOT, "tests", "golden", "fingertip50k_oracle.npz")
    if os.path.exists(gold_path):
        gold = np.load(gold_path)
        errs = {}
        for i, u in enumerate(r32["finals"]):
            key = f"u100_{3000 + i}"
            st = gold.get(f"status_{3000 + i}")
            if key in gold and st is not None and not np.any(st != 0):
                errs[str(3000 + i)] = float(np.abs(u - gold[key]).max() / np.abs(gold[key]).max())
        out["e_inf_vs_fp64_oracle"] = errs
    rl, kav = roofline(r32, 4)
    if rl:
        out["roofline"] = rl
        out["kernel_avg_us"] = kav
    if not args.no_fp64:
        r64 = run_batched(mesh, inds, "fp64", 1, 0, args.timing_every, track_latency=False)
        w64 = sum(r64["walls"])
        out["fp64_batched"] = {"solves_per_s": J / w64, "tet_updates_per_s": r64["tet_updates"] / w64,
                               "ms_per_step": w64 * 1e3, "failed_load_steps": r64["failed_steps"],
                               "floor_load_steps": r64["floor_steps"]}
        rl64, kav64 = roofline(r64, 8, kname="k_tile<double, LAW_NH>", peak=FP64_VECTOR_PEAK_TFLOPS)
        if rl64:
            out["fp64_batched"]["roofline"] = rl64
            out["fp64_batched"]["kernel_avg_us"] = kav64
        out["e_inf_fp32_vs_fp64"] = [float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))
                                     for a, b in zip(r32["finals"], r64["finals"])]
    if not args.no_single:
        s64 = run_single(mesh, inds[:args.single_jobs], "fp64")
        w = sum(s64["walls"])
        out["fp64_single_instance"] = {"solves_per_s": len(s64["walls"]) / w,
                                       "tet_updates_per_s": s64["tet_updates"] / w,
                                       "ms_per_job": w / len(s64["walls"]) * 1e3,
                                       "failed_load_steps": s64["failed_steps"],
                                       "jobs": len(s64["walls"])}
        out["speedup_vs_fp64_single_instance"] = out["value"] / out["fp64_single_instance"]["solves_per_s"]
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(mesh, inds[0], args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
