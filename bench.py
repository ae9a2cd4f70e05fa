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


def tile_bytes(info, word, hv_passes, el_passes, launches, n_act=None):
    """Algorithmic HBM bytes per launch of the tile kernel, averaged over
    `launches` launches that made hv_passes Hessian-vector passes and
    el_passes element passes in all (ideal reuse: every value read or written
    once per pass; the mesh constants once per launch).

    Shared per launch: packed local ids (4 B/tet), D_m^-1 and V (10 words per
    tet), the entry -> node map (4 B per entry).
    Hessian-vector pass, per job: reads of u, z, p_prev (9 words per node),
    write of the q partials (3 words per entry), the contact-block flags (1 B
    per eligible node) and the contact blocks of the nodes in contact (6
    words each; n_act of them, the job's final contact patch, which bounds
    the patch of every earlier step of the deepening indentation).
    Element pass, per job: reads of u and dx (6 words per node), write of the
    gradient + block partials (9 words per entry), contact node coordinates
    (3 doubles) and contact outputs (9 words) per eligible node.
    """
    n, m, nent, nc = info["n_nodes"], info["n_tets"], info["n_entries"], info["n_eligible"]
    na = nc if n_act is None else n_act
    shared = m * (4 + 10 * word) + 4 * nent
    hv = 9 * word * n + 3 * word * nent + nc + 6 * word * na
    el = 6 * word * n + 9 * word * nent + (24 + 9 * word + 1) * nc
    return shared + (hv_passes * hv + el_passes * el) / max(launches, 1)


def _plain(o):
    """JSON encoding of numpy scalars and arrays."""
    if isinstance(o, np.integer):
        return int(o)
    if isinstance(o, np.floating):
        return float(o)
    if isinstance(o, np.ndarray):
        return o.tolist()
    raise TypeError(type(o).__name__)


def emit(out):
    print(json.dumps(out, default=_plain), flush=True)


def progress(*a):
    print(*a, file=sys.stderr, flush=True)


def run_batched(mesh, inds, precision, timed_steps, warm_steps, timing_every=0, track_latency=True,
                material=(0.3e6, 0.45), groups=0, keep=(), round_steps=64):
    """Runs warm_steps untimed and timed_steps timed batches of the jobs
    `inds`; returns walls, latencies, counters (totals over the timed
    batches and per batch), kernel timing, and per-job results of the last
    timed batch: status, counters, displacement statistics and contact
    resultant for every job, and the final displacements of the job indices
    in `keep`. round_steps: solver steps per captured round (the host polls
    the jobs between rounds; the solve itself does not depend on it)."""
    from paper_2103_16747_amd import fem

    batch = fem.FemBatch(len(inds), precision)
    batch.set_option(fem.FEM_OPT_ROUND_STEPS, round_steps)
    if groups:
        batch.set_option(fem.FEM_OPT_GROUPS, groups)
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
    walls, lat, tu, failed, floor, hv, gp, ls = [], [], 0, 0, 0, 0, 0, 0
    per_batch_failed, per_batch_floor = [], []
    for _ in range(timed_steps):
        for j, ind in zip(jobs, inds):
            batch.restart_job(j, ind, *material)
        t0 = time.perf_counter()
        done_at = {}
        running = len(jobs)
        pending = list(jobs)
        while running:
            prev = running
            # completion times are taken every 128 solver steps
            running = batch.run(P, max_rounds=max(1, 128 // round_steps) if track_latency else 0)
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
        per_batch_failed.append(sum(i["steps_failed"] for i in infos))
        per_batch_floor.append(sum(i["steps_floor"] for i in infos))
        failed += per_batch_failed[-1]
        floor += per_batch_floor[-1]
        hv += sum(i["hv_products"] for i in infos)
        gp += sum(i["grad_passes"] for i in infos)
        ls += sum(i["ls_trials"] for i in infos)
        lat += list(done_at.values())
    timing = None
    if timing_every:
        timing = {k: batch.kernel_timing(k) + (batch.kernel_launches(k),)
                  for k in (fem.FEM_KERNEL_TILE, fem.FEM_KERNEL_NODE, fem.FEM_KERNEL_FINALIZE)}
        batch.set_kernel_timing(0)
    finals = {k: batch.displacements(jobs[k]) for k in keep}
    stats = [batch.job_info(j) for j in jobs]
    job_out = []
    for j in jobs:
        umax, umean = batch.displacement_stats(j)
        ids, _, _, Fr = batch.contact_patch(j)
        job_out.append({"status": batch.step_status(j), "umax": umax, "umean": umean, "F": Fr,
                        "patch": int(len(ids))})
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
            "failed_per_batch": per_batch_failed, "floor_per_batch": per_batch_floor,
            "outputs_ms_per_job": out_ms, "timing": timing, "hv_passes": hv, "grad_passes": gp, "ls_trials": ls,
            "layout": info, "finals": finals, "stats": stats, "jobs": job_out, "groups": groups}


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


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "fingertip50k_traffic.json")


def measured_traffic(groups):
    """HBM bytes per launch of the tile and node kernels from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE runs (copy-calibrated), or None when
    they are missing or were taken on a different kernel source or launch
    configuration (job groups per round)."""
    from paper_2103_16747_amd.profiling import kernel_source_hash

    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as f:
        t = json.load(f)
    if t.get("kernel_source_sha256") != kernel_source_hash() or t.get("groups") != groups:
        return None
    return {"tile": t.get("tile_bytes_per_dispatch"), "node": t.get("node_bytes_per_dispatch")}


FP64_VECTOR_PEAK_TFLOPS = 78.6      # 256 CU x 64 lanes x 2 x 2.4 GHz (FP64 vector)


def roofline(r, word, flops_per_tet=FLOPS_PER_TET, kname=None, peak=FP32_VECTOR_PEAK_TFLOPS, traffic=None):
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
    byts = tile_bytes(r["layout"], word, r["hv_passes"], r["grad_passes"], t["launches"], contact_nodes(r))
    if kname is None:
        kname = "k_tile<float, LAW_NH>" if word == 4 else "k_tile<double, LAW_NH>"
    out = {"bound": "alu", "kernel": kname, "achieved": achieved, "peak": peak,
           "unit": "TFLOP/s", "frac": achieved / peak, "traffic": traffic.get("tile") if traffic else None}
    if word == 4:
        out["frac_of_non_packed_peak"] = achieved / FP32_NONPACKED_PEAK_TFLOPS
    out.update({"avg_launch_us": t["avg_us"], "sampled_launches": t["sampled"], "launches": t["launches"],
                "flops_per_launch": per_launch,
                "tet_updates_per_launch": m * (r["hv_passes"] + r["grad_passes"]) / t["launches"],
                "hbm_model": {"algorithmic_bytes_per_launch": byts, "GB_per_s": byts / avg_s / 1e9,
                              "frac_of_hbm_peak": byts / avg_s / 1e9 / HBM_PEAK_GBS}})
    return out, {k: v["avg_us"] for k, v in per.items()}


def node_bytes(info, word, hv_passes, el_passes, launches, n_act=None):
    """Algorithmic HBM bytes per launch of the node kernel, averaged over
    `launches` launches that made hv_passes CG updates and followed el_passes
    element passes in all (ideal reuse: every value read or written once).

    Shared per launch: the node -> entry CSR (4 B per node and per entry),
    the contact index (4 B per node) and the fixed mask (1 B per node).
    CG update, per job and node: reads p, z, dx, r (12 words), the block
    inverse (6), the q partials (3 words per entry); writes p, dx, r, z (12);
    per contact-eligible node its contact-block flag (1 B), and the contact
    block (6 words) of the n_act nodes in contact (as for tile_bytes).
    After an element pass (Newton init; counted for every element pass, an
    upper bound for line-search trials, which read only g and dx): reads u
    and dx (6 words), the gradient and block partials (9 words per entry);
    writes u, g, the block inverse, r, z, p, dx (21 words); per eligible node
    the contact gradient and block (9 words).
    """
    n, nent, nc = info["n_nodes"], info["n_entries"], info["n_eligible"]
    na = nc if n_act is None else n_act
    shared = 4 * (n + 1) + 4 * nent + 4 * n + n
    cg = word * (30 * n + 3 * nent + 6 * na) + nc
    init = word * (27 * n + 9 * nent + 9 * nc)
    return shared + (hv_passes * cg + el_passes * init) / max(launches, 1)


def hbm_roofline(r, word, traffic=None):
    """HBM view of the solver: the node kernel (bound by memory) and the whole
    solver step (tile + node + finalize) as algorithmic bytes over time
    against the 8 TB/s peak, with the counter-measured bytes beside them
    where the committed rocprofv3 figures apply to this build."""
    from paper_2103_16747_amd import fem

    tm = r["timing"]
    if not tm:
        return None
    info = r["layout"]
    t_launch = tm[fem.FEM_KERNEL_TILE][2]
    n_cnt, n_ms, n_launch = tm[fem.FEM_KERNEL_NODE]
    node_avg_s = n_ms / max(n_cnt, 1) * 1e-3
    nb = node_bytes(info, word, r["hv_passes"], r["grad_passes"], n_launch, contact_nodes(r))
    tb = tile_bytes(info, word, r["hv_passes"], r["grad_passes"], t_launch, contact_nodes(r))
    jobs_steps = r["hv_passes"] + r["grad_passes"]
    fin_total = 8 * 3 * (info["n_tiles"] + ceil_div(info["n_eligible"], 256) + ceil_div(info["n_nodes"], 256)) * jobs_steps
    total = tb * t_launch + nb * n_launch + fin_total
    wall = sum(r["walls"])
    out = {"node_kernel": {"bound": "hbm", "kernel": "k_node", "achieved": nb / node_avg_s / 1e9, "peak": HBM_PEAK_GBS,
                           "unit": "GB/s", "frac": nb / node_avg_s / 1e9 / HBM_PEAK_GBS,
                           "algorithmic_bytes_per_launch": nb, "avg_launch_us": node_avg_s * 1e6,
                           "traffic": traffic.get("node") if traffic else None},
           "solver_step": {"bound": "hbm", "achieved": total / wall / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": total / wall / 1e9 / HBM_PEAK_GBS, "algorithmic_bytes": total,
                           "note": "tile + node + finalize algorithmic bytes of the timed batches over their wall time"}}
    if traffic and traffic.get("tile") and traffic.get("node"):
        meas = traffic["tile"] * t_launch + traffic["node"] * n_launch + fin_total
        out["solver_step"]["counter_bytes"] = meas
        out["solver_step"]["counter_frac"] = meas / wall / 1e9 / HBM_PEAK_GBS
    return out


def ceil_div(a, b):
    return (a + b - 1) // b


def contact_nodes(r):
    """Mean final contact-patch size of the timed batch's jobs (nodes whose
    contact block the Hessian-vector passes read), or None when unknown."""
    sizes = [j["patch"] for j in r.get("jobs", []) if "patch" in j]
    return float(np.mean(sizes)) if sizes else None


def _oracle_job(args):
    """One whole oracle job (FP64, one thread) of the batch workload; returns
    (seed, seconds, load steps, tet-updates)."""
    seed, steps_cap, seconds = args
    import oracle
    from paper_2103_16747_amd import workload as W

    mesh = W.fingertip_mesh(50000)
    ind = W.seat_on_mesh(W.random_indentation(seed), mesh)
    orc = oracle.Solver(mesh.X, mesh.tets, mesh.fixed, E=0.3e6, nu=0.45)
    u = np.zeros((mesh.n, 3))
    t0 = time.perf_counter()
    steps, passes = 0, 0
    for k in range(1, ind.steps + 1):
        orc.set_indenter(ind.kind, ind.shape, ind.R, ind.center(k), ind.k_penalty)
        u, info = orc.step(u)
        steps += 1
        passes += info["grad_passes"] + info["energy_passes"] + info["hv_products"]
        if steps >= steps_cap or (seconds and time.perf_counter() - t0 >= seconds):
            break
    return seed, time.perf_counter() - t0, steps, mesh.m * passes


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(seed0, all_seconds, single=True):
    """The FP64 oracle on the host: (a) one whole job (seed0, all 100 load
    steps) on one thread; (b) one job per host core (seeds seed0 + 1 ...), each
    process running its job's load steps for all_seconds, throughput summed
    over the processes (solves/s = load steps done / 100 / time)."""
    import multiprocessing as mp

    nproc = os.cpu_count() or 1
    cores = max(1, min(nproc, 16))
    out = {"kind": "oracle", "unit": "solves/s", "nproc": nproc, "cpu_model": cpu_model()}
    if single:
        progress("cpu oracle: one whole job on one thread")
        sd, el, steps, tu = _oracle_job((seed0, 100, 0))
        out["single_thread"] = {"solves_per_s": (steps / 100) / el, "seconds_per_job": el, "seed": sd,
                                "load_steps": steps, "tet_updates_per_s": tu / el}
    progress(f"cpu oracle: {cores} processes, {all_seconds:.0f} s each")
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        res = pool.map(_oracle_job, [(seed0 + 1 + i, 100, all_seconds) for i in range(cores)])
    wall = time.perf_counter() - t0
    rate = sum((st / 100) / el for _, el, st, _ in res)
    out.update({"value": rate, "cores": cores,
                "tet_updates_per_s": sum(tu / el for _, el, _, tu in res),
                "sample": f"FP64 oracle on {cores} host cores ({out['cpu_model']}, nproc {nproc}): one process per core, "
                          f"each on its own job of the batch workload (seeds {seed0 + 1}..{seed0 + cores}) for "
                          f"{all_seconds:.0f} s ({sum(st for _, _, st, _ in res)} load steps in all, "
                          f"{wall:.0f} s wall); solves/s = sum over processes of load steps / 100 / time"})
    return out


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
    """64 jobs at mixed resolution in one batch, tile shapes tuned per mesh
    and the round length for the mix by the autotuner, against the same 64
    jobs solved one at a time through the single-mesh API (FP32 path both);
    the tile kernel's roofline over the timed batch."""
    from paper_2103_16747_amd import autotune, fem

    meshes, jobs = uneven_jobs(64, 4000)
    mesh_list = [meshes[r] for r in RESOLUTIONS]
    tuned = autotune.tune(mesh_list, "fp32", cache=args.autotune_cache, log=progress)
    shape_of = dict(zip(RESOLUTIONS, tuned["shapes"]))
    progress(f"autotune: shapes {shape_of}, round length {tuned['chunk']}")
    batch = fem.FemBatch(len(jobs), "fp32")
    batch.set_option(fem.FEM_OPT_ROUND_STEPS, tuned["chunk"])
    mids = {}
    for r in RESOLUTIONS:
        autotune.apply_shape(batch, shape_of[r])
        mids[r] = batch.add_mesh(meshes[r].X, meshes[r].tets, meshes[r].fixed)
    layouts = {r: batch.mesh_info(mids[r]) for r in RESOLUTIONS}
    ids = [batch.add_job(mids[r], ind) for r, ind in jobs]
    batch.run()
    for j, (r, ind) in zip(ids, jobs):
        batch.restart_job(j, ind)
    batch.set_kernel_timing(args.timing_every)
    t0 = time.perf_counter()
    batch.run()
    wall = time.perf_counter() - t0
    infos = [batch.job_info(j) for j in ids]
    tm = {k: batch.kernel_timing(k) + (batch.kernel_launches(k),)
          for k in (fem.FEM_KERNEL_TILE, fem.FEM_KERNEL_NODE, fem.FEM_KERNEL_FINALIZE)}
    batch.close()
    progress(f"uneven batch: {len(jobs)} jobs in {wall:.2f} s")
    # the tile kernel's roofline: algorithmic flops of the passes the jobs made
    cnt, ms, launches = tm[fem.FEM_KERNEL_TILE]
    flops = sum(meshes[r].m * (i["hv_products"] * FLOPS_PER_TET["hv"] + i["grad_passes"] * FLOPS_PER_TET["element"])
                for (r, _), i in zip(jobs, infos))
    avg_s = ms / max(cnt, 1) * 1e-3
    achieved = flops / max(launches, 1) / avg_s / 1e12 if cnt else None
    rl = {"bound": "alu", "kernel": "k_tile<float, LAW_NH>", "achieved": achieved, "peak": FP32_VECTOR_PEAK_TFLOPS,
          "unit": "TFLOP/s", "frac": achieved / FP32_VECTOR_PEAK_TFLOPS if achieved else None, "traffic": None,
          "frac_of_non_packed_peak": achieved / FP32_NONPACKED_PEAK_TFLOPS if achieved else None,
          "avg_launch_us": avg_s * 1e6, "sampled_launches": cnt, "launches": launches}
    # every job one at a time through the single-mesh API (one fem_step per load step)
    solo_walls, solo_tu = [], 0
    for r in RESOLUTIONS:
        mine = [ind for rr, ind in jobs if rr == r]
        if mine:
            single = run_single(meshes[r], mine, "fp32")
            solo_walls += single["walls"]
            solo_tu += single["tet_updates"]
    solo = sum(solo_walls)
    tu = sum(i["tet_updates"] for i in infos)
    return {"metric": METRIC, "value": len(jobs) / wall, "unit": "solves/s", "n_gpus": 1, "steps": 1,
            "warmup": 1, "ms_per_step": wall * 1e3, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "uneven batch: 64 synthetic-fingertip jobs at 5k/20k/50k/120k tets (uniform mix), "
                                   "seeded indenters, 100 load steps each",
                       "mix": {str(r): sum(1 for rr, _ in jobs if rr == r) for r in RESOLUTIONS},
                       "autotuned": {"tile_shape_per_mesh": {str(r): shape_of[r] for r in RESOLUTIONS},
                                     "round_steps": tuned["chunk"]},
                       "layouts": {str(r): layouts[r] for r in RESOLUTIONS}},
            "tet_updates_per_s": tu / wall, "failed_load_steps": sum(i["steps_failed"] for i in infos),
            "floor_load_steps": sum(i["steps_floor"] for i in infos),
            "roofline": rl,
            "unbatched": {"solves_per_s": len(jobs) / solo, "tet_updates_per_s": solo_tu / solo, "wall_s": solo,
                          "jobs": len(solo_walls),
                          "note": "all 64 jobs one at a time through the single-mesh API, FP32 path"},
            "speedup_vs_unbatched": solo / wall,
            "autotune": {"per_mesh": tuned["per_mesh"], "round_length_table": tuned["table"]}}


def bench_serving(args):
    """Poisson streams of mixed-resolution jobs through the serving loop
    (admission by HBM footprint, continuous batching): per arrival rate,
    args.warmup_requests requests warm the server up and the next
    args.requests are measured (p50/p99 latency from arrival to the result
    on the host, solves/s); against the one-at-a-time FP64 path timed on a
    sample of the same jobs."""
    from paper_2103_16747_amd import fem, workload as W
    from paper_2103_16747_amd.serve import IndentationServer, Request, latency_summary

    warm = args.warmup_requests
    meshes, jobs = uneven_jobs(warm + args.requests, 5000)
    keyed = {str(r): meshes[r] for r in RESOLUTIONS}
    out = {"metric": METRIC, "unit": "ms", "n_gpus": 1, "higher_is_better": False, "data": "synthetic",
           "dtype": "f32", "config": {"workload": f"serving: Poisson arrivals of {warm} warm-up and {args.requests} "
                                                  "measured mixed-resolution fingertip jobs (5k-120k tets) per rate, "
                                                  "100 load steps each",
                                      "hbm_budget_GiB": 64}, "rates": {}}
    for rate in [float(x) for x in args.rates.split(",")]:
        arrivals = W.poisson_arrivals(int(rate * 1000), rate, len(jobs))
        reqs = [Request(i, float(t), str(r), ind) for i, (t, (r, ind)) in enumerate(zip(arrivals, jobs))]
        batch = fem.FemBatch(len(jobs), "fp32")
        srv = IndentationServer(batch, keyed, hbm_budget=64 << 30, max_jobs=len(jobs), rounds_per_poll=2)
        res = srv.serve(reqs, timeout=1500, progress=progress)
        summ = latency_summary(res, skip=warm)
        summ["peak_running"] = srv.stats.peak_running
        summ["warmup_requests"] = warm
        out["rates"][str(rate)] = summ
        batch.close()
        progress(f"serving rate {rate}: p50 {summ['p50_ms']:.0f} ms p99 {summ['p99_ms']:.0f} ms "
                 f"{summ['solves_per_s']:.1f} solves/s")
    # one-at-a-time FP64 reference on a sample of the measured jobs, per resolution
    ref = {}
    for r in RESOLUTIONS:
        sample = [ind for rr, ind in jobs[warm:] if rr == r][:args.fp64_sample]
        if sample:
            w = run_single(meshes[r], sample, "fp64")["walls"]
            ref[str(r)] = sum(w) / len(w)
    measured = [r for r, _ in jobs[warm:]]
    mean_one = sum(ref[str(r)] for r in measured) / len(measured)
    out["fp64_one_at_a_time"] = {"solves_per_s": 1.0 / mean_one, "mean_s_per_job": ref,
                                 "note": f"the first {args.fp64_sample} measured jobs of each resolution one at a time "
                                         "(single-mesh API, FP64), weighted by the stream's resolution mix"}
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
            "tet_updates_per_s": tu / wall, "failed_load_steps_per_batch": failed / K,
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
           "failed_load_steps_per_batch": float(np.mean(r["failed_per_batch"])),
           "floor_load_steps_per_batch": float(np.mean(r["floor_per_batch"])),
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


STRAT_GOLD = os.path.join(ROOT, "tests", "golden", "fingertip50k_stratified_oracle.npz")
SUMM_GOLD = os.path.join(ROOT, "tests", "golden", "fingertip50k_batch_summary.npz")


def stratified_keep(J):
    """Job indices (seed - 3000) of the stored stratified oracle results."""
    if not os.path.exists(STRAT_GOLD):
        return []
    return [int(x) - 3000 for x in np.load(STRAT_GOLD)["seeds"] if int(x) - 3000 < J]


def accuracy(r, bound):
    """Per-instance agreement of the last timed batch with the stored FP64
    oracle results: e_inf at load step 100 for the stratified seeds (full
    fields), and for every job the relative error of max|u|, mean|u| and the
    contact resultant at step 100 (where the oracle and the device both
    ended the step converged or at the floor); the device's capped steps with
    the oracle's status at the same steps."""
    if not (os.path.exists(STRAT_GOLD) and os.path.exists(SUMM_GOLD)):
        return None
    strat, summ = np.load(STRAT_GOLD), np.load(SUMM_GOLD)
    row = {int(x): i for i, x in enumerate(summ["seeds"])}
    out = {"bound": bound, "stratified_e_inf_step100": {}, "capped_steps": {}}
    for k, u in r["finals"].items():
        seed = 3000 + k
        st = r["jobs"][k]["status"]
        if summ["status"][row[seed]][99] == 0 and st[99] >= 0:
            ref = strat[f"u100_{seed}"]
            out["stratified_e_inf_step100"][str(seed)] = float(np.abs(u - ref).max() / np.abs(ref).max())
    errs, above = [], []
    for k, job in enumerate(r["jobs"]):
        seed = 3000 + k
        i = row.get(seed)
        if i is None:
            continue
        st = job["status"]
        capped = [int(q) + 1 for q in np.nonzero(st < 0)[0]]
        if capped:
            out["capped_steps"][str(seed)] = [[q, int(summ["status"][i][q - 1])] for q in capped]
        if summ["status"][i][99] != 0 or st[99] < 0:
            continue
        F = summ["F"][i][99]
        e = max(abs(job["umax"] - summ["umax"][i][99]) / summ["umax"][i][99],
                abs(job["umean"] - summ["umean"][i][99]) / summ["umean"][i][99],
                float(np.abs(job["F"] - F).max() / max(np.abs(F).max(), 1e-300)))
        errs.append(e)
        if e > bound:
            above.append([seed, e])
    out["all_jobs_step100"] = {"jobs_compared": len(errs), "max_rel_err": max(errs) if errs else None,
                               "median_rel_err": float(np.median(errs)) if errs else None,
                               "within_bound": sum(e <= bound for e in errs), "above_bound": above,
                               "quantities": "max|u|, mean|u| and contact resultant, relative to the oracle's"}
    out["capped_steps_note"] = "per seed: [load step, oracle status at that step (0 converged, -6 capped)]"
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2, help="timed batches")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--jobs", type=int, default=256)
    ap.add_argument("--single-jobs", type=int, default=3, help="jobs timed one at a time on the FP64 path")
    ap.add_argument("--cpu-seconds", type=float, default=20.0, help="CPU baseline: seconds per process, all cores")
    ap.add_argument("--no-cpu-single", action="store_true", help="CPU baseline: skip the whole single-thread job")
    ap.add_argument("--groups", type=int, default=0, help="job groups per round (0 or 1: one, 2: two)")
    ap.add_argument("--autotune-cache", default=None, help="uneven: JSON cache of the autotuner's results")
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
    ap.add_argument("--rates", default="10,20,50,100,200,500", help="serving: arrival rates (req/s)")
    ap.add_argument("--requests", type=int, default=2000, help="serving: measured requests per rate")
    ap.add_argument("--warmup-requests", type=int, default=200, help="serving: warm-up requests per rate")
    ap.add_argument("--fp64-sample", type=int, default=8, help="serving: FP64 one-at-a-time jobs per resolution")
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
        emit(bench_uneven(args))
        return
    if args.config == "serving":
        emit(bench_serving(args))
        return
    if args.config == "dynamic":
        emit(bench_dynamic(args))
        return
    if args.config in VARIANTS:
        emit(bench_variant(args, args.config))
        return
    mesh = W.fingertip_mesh(50000)
    inds = [W.seat_on_mesh(W.random_indentation(3000 + i), mesh) for i in range(args.jobs)]

    keep = stratified_keep(args.jobs)
    torch.cuda.synchronize()
    r32 = run_batched(mesh, inds, "fp32", args.steps, args.warmup, args.timing_every, groups=args.groups, keep=keep)
    torch.cuda.synchronize()
    groups_used = 2 if args.groups == 2 else 1
    traffic = measured_traffic(groups_used)
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
        "load_steps_per_batch": J * 100,
        "failed_load_steps_per_batch": float(np.mean(r32["failed_per_batch"])),
        "floor_load_steps_per_batch": float(np.mean(r32["floor_per_batch"])),
        "cg_iters_per_job": float(np.mean([s["cg_iters"] for s in r32["stats"]])),
        "outputs_ms_per_job": r32["outputs_ms_per_job"],
        "newton_iters_per_job": float(np.mean([s["newton_iters"] for s in r32["stats"]])),
        "job_groups_per_round": groups_used,
    }
    acc = accuracy(r32, 1e-4)
    if acc:
        out["accuracy_vs_fp64_oracle"] = acc
    rl, kav = roofline(r32, 4, traffic=traffic)
    if rl:
        out["roofline"] = rl
        out["kernel_avg_us"] = kav
        out["roofline_hbm"] = hbm_roofline(r32, 4, traffic)
    if not args.no_fp64:
        r64 = run_batched(mesh, inds, "fp64", 1, 0, args.timing_every, track_latency=False, groups=args.groups,
                          keep=keep)
        w64 = sum(r64["walls"])
        out["fp64_batched"] = {"solves_per_s": J / w64, "tet_updates_per_s": r64["tet_updates"] / w64,
                               "ms_per_step": w64 * 1e3, "failed_load_steps_per_batch": r64["failed_steps"],
                               "floor_load_steps_per_batch": r64["floor_steps"]}
        acc64 = accuracy(r64, 1e-8)
        if acc64:
            out["fp64_batched"]["accuracy_vs_fp64_oracle"] = acc64
        rl64, kav64 = roofline(r64, 8, kname="k_tile<double, LAW_NH>", peak=FP64_VECTOR_PEAK_TFLOPS)
        if rl64:
            out["fp64_batched"]["roofline"] = rl64
            out["fp64_batched"]["kernel_avg_us"] = kav64
        out["e_inf_fp32_vs_fp64"] = {str(3000 + k): float(np.abs(r32["finals"][k] - b).max() /
                                                          max(np.abs(b).max(), 1e-300))
                                     for k, b in r64["finals"].items()}
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
        out["cpu_baseline"] = cpu_baseline(3000, args.cpu_seconds, single=not args.no_cpu_single)
    emit(out)


if __name__ == "__main__":
    main()
