"""Admission and completion logic of the serving loop, on the CPU with a
fake engine that finishes each job after a set number of rounds."""
import numpy as np
import pytest

from paper_2103_16747_amd.serve import IndentationServer, Request, latency_summary


class FakeMesh:
    def __init__(self, n):
        self.X = np.zeros((n, 3))
        self.tets = np.zeros((1, 4), dtype=np.int32)
        self.fixed = np.zeros(n, dtype=np.uint8)


class FakeEngine:
    """Jobs finish after `indentation.steps` rounds; tracks allocations."""

    def __init__(self, capacity):
        self.capacity = capacity
        self.meshes = []
        self.slots = {}          # slot -> [mesh_id, rounds_left, done]
        self.events = []

    def add_mesh(self, X, tets, fixed):
        self.meshes.append(X.shape[0])
        return len(self.meshes) - 1

    def job_footprint(self, mid):
        return 1000 * self.meshes[mid]

    def add_job(self, mid, ind, E, nu):
        free = [s for s in range(self.capacity) if s not in self.slots]
        assert free, "engine over capacity"
        s = free[0]
        self.slots[s] = [mid, ind.steps, False]
        self.events.append(("add", s))
        return s

    def restart_job(self, s, ind, E, nu):
        assert s in self.slots and self.slots[s][2]
        self.slots[s][1:] = [ind.steps, False]
        self.events.append(("restart", s))

    def remove_job(self, s):
        del self.slots[s]
        self.events.append(("remove", s))

    def run(self, params, max_rounds):
        for _ in range(max_rounds):
            for v in self.slots.values():
                if not v[2]:
                    v[1] -= 1
                    if v[1] <= 0:
                        v[2] = True

    def job_info(self, s):
        return {"done": int(self.slots[s][2]), "status": 0, "steps_ok": 1, "steps_failed": 0, "cg_iters": 7,
                "tet_updates": 11}

    def displacements(self, s):
        return np.zeros((3, 3))


class Ind:
    def __init__(self, steps):
        self.steps = steps


def requests(specs):
    return [Request(i, t, mesh, Ind(steps)) for i, (t, mesh, steps) in enumerate(specs)]


def test_budget_limits_concurrency_and_all_complete():
    eng = FakeEngine(capacity=8)
    srv = IndentationServer(eng, {"a": FakeMesh(10)}, hbm_budget=2 * 10000, max_jobs=8, rounds_per_poll=1)
    res = srv.serve(requests([(0.0, "a", 3)] * 5), timeout=10)
    assert [r.rid for r in res] == list(range(5))
    assert srv.stats.peak_running <= 2 and srv.stats.peak_bytes <= 20000
    assert srv.stats.allocated == 2 and srv.stats.restarted_in_place == 3
    assert all(r.done >= r.admitted >= r.arrival for r in res)
    s = latency_summary(res)
    assert s["completed"] == 5 and s["p99_ms"] >= s["p50_ms"]


def test_idle_slot_of_other_mesh_is_released():
    eng = FakeEngine(capacity=4)
    meshes = {"small": FakeMesh(10), "big": FakeMesh(20)}
    srv = IndentationServer(eng, meshes, hbm_budget=25000, max_jobs=4, rounds_per_poll=1)
    res = srv.serve(requests([(0.0, "small", 2), (0.0, "small", 2), (0.05, "big", 2)]), timeout=10)
    assert len(res) == 3
    assert srv.stats.released >= 1
    assert ("remove", 0) in eng.events or ("remove", 1) in eng.events


def test_job_slot_count_cap():
    eng = FakeEngine(capacity=1)
    srv = IndentationServer(eng, {"a": FakeMesh(1)}, hbm_budget=10 ** 9, max_jobs=1, rounds_per_poll=1)
    res = srv.serve(requests([(0.0, "a", 2), (0.0, "a", 2), (0.0, "a", 2)]), timeout=10)
    assert len(res) == 3 and srv.stats.peak_running == 1


def test_request_that_never_fits_is_rejected():
    """A job whose footprint exceeds the whole budget is refused at arrival
    with an error result (no spinning), and the others are still served."""
    from paper_2103_16747_amd.serve import REJECTED_FOOTPRINT

    eng = FakeEngine(capacity=2)
    srv = IndentationServer(eng, {"a": FakeMesh(100), "b": FakeMesh(1)}, hbm_budget=5000, max_jobs=2,
                            rounds_per_poll=1)
    res = srv.serve(requests([(0.0, "a", 1), (0.0, "b", 2), (0.01, "a", 1)]), timeout=5)
    assert [r.status for r in res] == [REJECTED_FOOTPRINT, 0, REJECTED_FOOTPRINT]
    assert srv.stats.rejected == 2 and srv.stats.admitted == 1
    assert not any(e[0] == "add" and eng.slots.get(e[1], [None])[0] == 0 for e in eng.events)
    assert latency_summary(res)["completed"] == 1


def test_latency_summary_skips_warmup_requests():
    from paper_2103_16747_amd.serve import Result, latency_summary

    res = [Result(i, "m", float(i), float(i), float(i) + (10.0 if i < 2 else 1.0), 0, 1, 0, 0, 0) for i in range(6)]
    all_ = latency_summary(res)
    meas = latency_summary(res, skip=2)
    assert all_["completed"] == 6 and meas["completed"] == 4
    assert meas["max_ms"] == 1000.0 and all_["max_ms"] == 10000.0
    assert meas["solves_per_s"] == 4 / (6.0 - 2.0)
