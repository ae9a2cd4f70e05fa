#!/usr/bin/env python3
"""Benchmark of the indentation solve on one MI355X.

A step is one complete indentation job: a seeded rigid indenter (sphere,
cylinder, box or ring; random surface point, tilt and depth) pressed into the
synthetic 50k-tet fingertip in 100 quasi-static load steps, each solved by
Newton + matrix-free block-Jacobi PCG on the device, starting from rest. The
mesh is resident in HBM before the timed region; every timed step runs a
different seed.

Prints one JSON line: solves/s of the FP32 path (FP32 element math and CG
vectors, FP64 reductions) with tet-updates/s, per-solve latency percentiles,
the plain FP64 path on the same seeds, the roofline of the Hessian-vector
kernel (event-timed on the library's stream during the timed region), and the
FP64 CPU oracle timed on a bounded sample of the same workload.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0
METRIC = "FEM indentation solves/s + tet-updates/s, FP32 vs FP64 path; p50/p99 latency"


def hv_bytes_per_launch(m, n, nc, word):
    """Algorithmic HBM bytes of one Hessian-vector launch: per tet the four
    node ids (16 B), D_m^-1 (9 words), V, the cached F^-1 (9 words) and
    mu - lam ln J; per node the reads of z and p_prev (6 words) and the
    read-modify-write of q (6 words); per contact-eligible node its id and
    contact block (6 words)."""
    return m * (16 + 20 * word) + n * 12 * word + nc * (4 + 6 * word)


def run_solves(mesh, inds, precision, stream, timing_every=0):
    from paper_2103_16747_amd import fem

    dev = fem.FemMesh(mesh.X, mesh.tets, mesh.fixed, precision=precision, device=0, stream=stream)
    dev.set_material(0.3e6, 0.45, 1100.0)
    zeros = np.zeros((mesh.n, 3))
    return dev, zeros


def solve_one(dev, zeros, ind):
    dev.set_displacements(zeros)
    tet_updates = 0
    statuses = []
    for k in range(1, ind.steps + 1):
        dev.set_indenter(ind.kind, ind.shape, ind.R, ind.center(k), ind.k_penalty)
        info = dev.step()
        tet_updates += info["tet_updates"]
        statuses.append(info["status"])
    return tet_updates, statuses


def time_path(mesh, warm, timed, precision, torch, timing_every):
    from paper_2103_16747_amd import fem

    stream = torch.cuda.Stream()
    dev, zeros = run_solves(mesh, timed, precision, stream)
    for ind in warm:
        solve_one(dev, zeros, ind)
    if timing_every:
        dev.set_kernel_timing(timing_every)
    torch.cuda.synchronize()
    lat, tu, bad = [], 0, 0
    finals = []
    t0 = time.perf_counter()
    for ind in timed:
        s0 = time.perf_counter()
        n_tu, st = solve_one(dev, zeros, ind)
        lat.append(time.perf_counter() - s0)
        tu += n_tu
        bad += sum(1 for s in st if s != 0)
        finals.append(dev.displacements())
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    timing = None
    if timing_every:
        timing = {k: dev.kernel_timing(k) for k in (fem.FEM_KERNEL_HV, fem.FEM_KERNEL_CG_UPDATE, fem.FEM_KERNEL_ELEMENT)}
        dev.set_kernel_timing(0)
    n_elig = dev.info()["n_eligible"]
    dev.close()
    return {"wall": wall, "lat": lat, "tet_updates": tu, "failed_steps": bad, "finals": finals, "timing": timing,
            "n_eligible": n_elig}


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
    el = time.perf_counter() - t0
    return {"value": (steps / ind.steps) / el, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "tet_updates_per_s": mesh.m * passes / el,
            "sample": f"FP64 oracle, one thread, first {steps} of {ind.steps} load steps of seed {ind.seed} "
                      f"on the {mesh.m}-tet fingertip ({el:.1f} s); solves/s = ({steps}/{ind.steps}) / time"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="timed indentation solves")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--timing-every", type=int, default=4)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this solver runs each indentation job on a single MI355X and has "
              "no multi-GPU path; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2103_16747_amd import fem, workload as W

    assert torch.cuda.is_available(), "no GPU visible"
    torch.cuda.set_device(0)
    fem.load()
    mesh = W.fingertip_mesh(50000)
    timed = [W.seat_on_mesh(W.random_indentation(W.instance_seed(2, i)), mesh) for i in range(1, args.steps + 1)]
    warm = [W.seat_on_mesh(W.random_indentation(W.instance_seed(2, 900 + i)), mesh) for i in range(args.warmup)]

    r32 = time_path(mesh, warm, timed, "fp32", torch, args.timing_every)
    r64 = None if args.no_fp64 else time_path(mesh, warm, timed, "fp64", torch, 0)

    K = args.steps
    value = K / r32["wall"]
    lat_ms = np.array(r32["lat"]) * 1e3
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": r32["wall"] / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "synthetic fingertip, 50k tets, one seeded indenter per solve, 100 quasi-static load steps",
            "mesh_tets": mesh.m, "mesh_nodes": mesh.n, "contact_eligible_nodes": r32["n_eligible"],
            "seeds": [ind.seed for ind in timed],
            "indenters": [W.KIND_NAMES[ind.kind] for ind in timed],
            "precision": "fp32 element math and CG vectors; fp64 dots, norms, energies, Newton test, contact",
            "solver": "Newton + block-Jacobi PCG (matrix-free), Armijo line search, exact contact Hessian",
        },
        "tet_updates_per_s": r32["tet_updates"] / r32["wall"],
        "latency_ms": {"p50": float(np.percentile(lat_ms, 50)), "p99": float(np.percentile(lat_ms, 99)),
                       "mode": "one job at a time"},
        "failed_load_steps": r32["failed_steps"],
    }
    if r64 is not None:
        errs = [float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)) for a, b in zip(r32["finals"], r64["finals"])]
        out["fp64_path"] = {"solves_per_s": K / r64["wall"], "tet_updates_per_s": r64["tet_updates"] / r64["wall"],
                            "ms_per_step": r64["wall"] / K * 1e3, "failed_load_steps": r64["failed_steps"]}
        out["e_inf_fp32_vs_fp64_path"] = errs
    tm = r32["timing"]
    if tm and tm[fem.FEM_KERNEL_HV][0] > 0:
        cnt, ms = tm[fem.FEM_KERNEL_HV]
        avg_s = ms / cnt * 1e-3
        byts = hv_bytes_per_launch(mesh.m, mesh.n, r32["n_eligible"], 4)
        achieved = byts / avg_s / 1e9
        out["roofline"] = {"bound": "hbm", "kernel": "k_cg_hv<float>", "achieved": achieved, "peak": HBM_PEAK_GBS,
                           "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                           "avg_launch_us": avg_s * 1e6, "sampled_launches": cnt,
                           "algorithmic_bytes_per_launch": byts,
                           "bytes_per_tet_update": byts / mesh.m}
        out["kernel_avg_us"] = {name: (tm[k][1] / tm[k][0] * 1e3 if tm[k][0] else None)
                                for name, k in (("hv", fem.FEM_KERNEL_HV), ("cg_update", fem.FEM_KERNEL_CG_UPDATE),
                                                ("element", fem.FEM_KERNEL_ELEMENT))}
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(mesh, timed[0], args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
