"""CPU checks of bench.py's contract: it refuses more than one GPU before
touching the device, its roofline arithmetic, and the gating of the committed
HBM traffic figure on the kernel source it was measured on."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def fake_run(timing, hv, grad, word_tets=49584):
    return {"timing": timing, "hv_passes": hv, "grad_passes": grad,
            "layout": {"n_tets": word_tets, "n_nodes": 11249, "n_entries": 21652, "n_eligible": 3757}}


def test_roofline_arithmetic():
    # 100 tile launches, 10 of them sampled for 1 ms in all (100 us each)
    r = fake_run({0: (10, 1.0, 100), 1: (10, 0.5, 100), 2: (10, 0.05, 100)}, hv=900, grad=100)
    rl, kav = bench.roofline(r, 4, traffic={"tile": 1.0e8, "node": 2.0e8})
    flops = 49584 * (900 * bench.FLOPS_PER_TET["hv"] + 100 * bench.FLOPS_PER_TET["element"]) / 100
    assert rl["flops_per_launch"] == pytest.approx(flops)
    assert rl["avg_launch_us"] == pytest.approx(100.0)
    assert rl["achieved"] == pytest.approx(flops / 100e-6 / 1e12)
    assert rl["frac"] == pytest.approx(rl["achieved"] / 157.3)
    assert rl["frac_of_non_packed_peak"] == pytest.approx(rl["achieved"] / 78.6)
    assert rl["bound"] == "alu" and rl["unit"] == "TFLOP/s" and rl["traffic"] == 1.0e8
    assert kav == {"tile": pytest.approx(100.0), "node": pytest.approx(50.0), "finalize": pytest.approx(5.0)}
    # the FP64 instance: its own peak, no FP32 traffic figure
    rl64, _ = bench.roofline(r, 8, kname="k_tile<double, LAW_NH>", peak=bench.FP64_VECTOR_PEAK_TFLOPS)
    assert rl64["frac"] == pytest.approx(rl64["achieved"] / 78.6) and rl64["traffic"] is None
    # no sampled launches: no roofline
    assert bench.roofline(fake_run(None, 1, 1), 4) == (None, None)


def test_corotational_flop_counts():
    assert bench.FLOPS_PER_TET_CR == {"hv": round(223 + 3 + 83 * 2.2 + 102 + 184),
                                      "element": round(305 + 3 + 83 * 2.2 + 243 + 81)}


def test_traffic_figure_follows_the_kernel_source_and_launch(monkeypatch, tmp_path):
    from paper_2103_16747_amd import profiling

    f = tmp_path / "traffic.json"
    rec = {"kernel_source_sha256": profiling.kernel_source_hash(), "groups": 2,
           "tile_bytes_per_dispatch": 123.0, "node_bytes_per_dispatch": 456.0}
    f.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.measured_traffic(2) == {"tile": 123.0, "node": 456.0}
    assert bench.measured_traffic(1) is None          # taken with another launch configuration
    f.write_text(json.dumps(dict(rec, kernel_source_sha256="0" * 64)))
    assert bench.measured_traffic(2) is None          # taken on other kernels


def test_node_bytes_model():
    info = {"n_nodes": 100, "n_entries": 200, "n_eligible": 10, "n_tets": 300, "n_tiles": 1}
    shared = 4 * 101 + 4 * 200 + 4 * 100 + 100
    # one CG update of one job per launch, FP32: 30 words per node, 3 per entry, a flag byte per
    # eligible node and 6 words per node in contact (all eligible ones when the patch is unknown)
    assert bench.node_bytes(info, 4, 1, 0, 1) == pytest.approx(shared + 4 * (30 * 100 + 3 * 200 + 6 * 10) + 10)
    assert bench.node_bytes(info, 4, 1, 0, 1, n_act=3) == pytest.approx(shared + 4 * (30 * 100 + 3 * 200 + 6 * 3) + 10)
    # one element pass followed by a Newton init, FP64
    assert bench.node_bytes(info, 8, 0, 1, 1) == pytest.approx(shared + 8 * (27 * 100 + 9 * 200 + 9 * 10))


def test_tile_bytes_model():
    info = {"n_nodes": 100, "n_entries": 200, "n_eligible": 10, "n_tets": 300, "n_tiles": 1}
    shared = 300 * (4 + 10 * 4) + 4 * 200
    # one Hessian-vector pass: u, z, p_prev per node, q partials per entry, flags, blocks in contact
    assert bench.tile_bytes(info, 4, 1, 0, 1, n_act=2) == pytest.approx(shared + 4 * (9 * 100 + 3 * 200 + 6 * 2) + 10)
    # one element pass: u, dx per node, 9 partials per entry, contact coordinates, outputs and flag
    assert bench.tile_bytes(info, 4, 0, 1, 1) == pytest.approx(shared + 4 * (6 * 100 + 9 * 200) + (24 + 36 + 1) * 10)


def test_contact_nodes_mean_patch():
    assert bench.contact_nodes({"jobs": [{"patch": 10}, {"patch": 30}]}) == pytest.approx(20.0)
    assert bench.contact_nodes({"jobs": []}) is None


def test_hbm_roofline_arithmetic():
    r = fake_run({0: (10, 1.0, 100), 1: (10, 0.5, 100), 2: (10, 0.05, 100)}, hv=900, grad=100)
    r["layout"]["n_tiles"] = 97
    r["walls"] = [0.1]
    h = bench.hbm_roofline(r, 4, traffic={"tile": 1.0e8, "node": 2.0e8})
    nb = bench.node_bytes(r["layout"], 4, 900, 100, 100)
    assert h["node_kernel"]["achieved"] == pytest.approx(nb / 50e-6 / 1e9)
    assert h["node_kernel"]["frac"] == pytest.approx(h["node_kernel"]["achieved"] / 8000.0)
    assert h["node_kernel"]["traffic"] == 2.0e8
    tb = bench.tile_bytes(r["layout"], 4, 900, 100, 100)
    assert h["solver_step"]["algorithmic_bytes"] > 100 * (tb + nb)
    assert h["solver_step"]["frac"] == pytest.approx(h["solver_step"]["algorithmic_bytes"] / 0.1 / 8e12)
    assert h["solver_step"]["counter_frac"] > h["solver_step"]["frac"] * 0 and "counter_bytes" in h["solver_step"]


def test_kernel_source_hash_ignores_comments():
    from paper_2103_16747_amd.profiling import kernel_source_hash

    a = "int f() {\n  return 1; // one\n}\n"
    b = "// header\nint f() {\n\n  return 1;\n}\n"
    assert kernel_source_hash(a) == kernel_source_hash(b)
    assert kernel_source_hash(a) != kernel_source_hash(a.replace("1", "2"))


def test_line_encodes_numpy_values(capsys):
    import numpy as np

    bench.emit({"a": np.int64(3), "b": np.float32(1.5), "c": np.arange(2), "d": [np.int32(1)]})
    assert json.loads(capsys.readouterr().out) == {"a": 3, "b": 1.5, "c": [0, 1], "d": [1]}
