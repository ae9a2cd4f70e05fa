"""CPU checks of the autotuner's selection and cache (timing stubbed: no GPU)."""
import json

from paper_2103_16747_amd import autotune, workload as W


def fake_timer(calls):
    """Deterministic timing: per mesh the (384, 256) shape is fastest on the
    larger mesh and (128, 128) on the smaller; round length 16 is fastest."""
    def timer(meshes, jobs, precision, shapes, chunk):
        calls.append((tuple(m.m for m in meshes), tuple(shapes), chunk))
        tets, nodes = shapes[0]
        big = meshes[0].m > 500
        best = (384, 256) if big else (128, 128)
        wall = 1.0 + 0.1 * (abs(tets - best[0]) + abs(nodes - best[1])) / 128 + 0.05 * abs(chunk - 16) / 8
        return wall, 1.0e6
    return timer


def test_per_mesh_shapes_and_cache_round_trip(monkeypatch, tmp_path):
    calls = []
    monkeypatch.setattr(autotune, "_time_config", fake_timer(calls))
    monkeypatch.setattr(autotune, "_short_jobs", lambda mesh, count, seed0, steps: [None] * count)
    small, big = W.block_mesh((2, 2, 2)), W.block_mesh((6, 6, 6))
    cache = str(tmp_path / "tune.json")
    out = autotune.tune([small, big], "fp32", cache=cache)
    assert out["shapes"] == [(128, 128), (384, 256)]
    assert out["chunk"] == 16
    n_first = len(calls)
    assert n_first == 2 * len(autotune.SHAPE_CANDIDATES) + len(autotune.CHUNK_CANDIDATES)
    known = json.load(open(cache))
    assert autotune.mesh_key(small, "fp32") in known["meshes"]
    assert autotune.mesh_key(big, "fp32") in known["meshes"]
    # a second call reads everything from the cache
    again = autotune.tune([small, big], "fp32", cache=cache)
    assert len(calls) == n_first
    assert again["shapes"] == out["shapes"] and again["chunk"] == out["chunk"]
    # another precision or another mesh is timed anew; a known mesh is not
    autotune.tune_mesh(big, "fp64", cache=cache)
    assert len(calls) == n_first + len(autotune.SHAPE_CANDIDATES)
    other = W.block_mesh((3, 3, 3))
    autotune.tune([small, other], "fp32", cache=cache)
    assert len(calls) == n_first + 2 * len(autotune.SHAPE_CANDIDATES) + len(autotune.CHUNK_CANDIDATES)


def test_mesh_key_follows_the_mesh():
    a, b = W.block_mesh((2, 2, 2)), W.block_mesh((2, 2, 2))
    assert autotune.mesh_key(a, "fp32") == autotune.mesh_key(b, "fp32")
    assert autotune.mesh_key(a, "fp32") != autotune.mesh_key(a, "fp64")
    b.X = b.X * 1.001
    assert autotune.mesh_key(a, "fp32") != autotune.mesh_key(b, "fp32")


def test_candidates_within_library_limits():
    for tets, nodes in autotune.SHAPE_CANDIDATES:
        assert 64 <= tets <= 512 and 16 <= nodes <= 256
    assert all(1 <= c <= 64 for c in autotune.CHUNK_CANDIDATES)
