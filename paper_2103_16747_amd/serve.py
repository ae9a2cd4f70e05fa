"""Serving loop for indentation jobs on one GPU (continuous batching).

Requests (a mesh, a material and a seeded indentation) arrive over time. A
request is admitted as soon as a job slot and its HBM footprint are
available: a finished job's slot on the same mesh is restarted in place (no
allocation), otherwise a new slot is allocated if the footprint budget
allows, otherwise an idle slot of another mesh is released first. All
admitted jobs advance together in rounds of the batch engine, so a job that
arrives while others are mid-solve starts at the next round and its work
overlaps theirs on the device; each job's state (mesh, displacements, solver
state) stays resident from admission to completion. Latency is measured from
arrival to the result being readable on the host.

The engine is any object with the FemBatch interface (add_mesh, add_job,
restart_job, remove_job, run, job_info, displacements, job_footprint), so
the admission logic is testable without a GPU.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    rid: int
    arrival: float              # seconds from the start of serving
    mesh: str                   # key into the server's meshes
    indentation: object         # workload.Indentation
    E: float = 0.3e6
    nu: float = 0.45


@dataclass
class Result:
    rid: int
    mesh: str
    arrival: float
    admitted: float
    done: float
    status: int
    steps_ok: int
    steps_failed: int
    cg_iters: int
    tet_updates: int
    u: np.ndarray | None = None

    @property
    def latency(self) -> float:
        return self.done - self.arrival


# Result.status of a request refused at arrival: its job's device footprint
# exceeds the whole HBM budget, so it could never be admitted (the C ABI's
# out-of-memory code).
REJECTED_FOOTPRINT = -3


@dataclass
class ServerStats:
    rejected: int = 0
    admitted: int = 0
    restarted_in_place: int = 0
    allocated: int = 0
    released: int = 0
    waits_for_memory: int = 0
    rounds: int = 0
    peak_bytes: int = 0
    peak_running: int = 0
    extra: dict = field(default_factory=dict)


class IndentationServer:
    def __init__(self, engine, meshes: dict, hbm_budget: int, max_jobs: int, params=None, rounds_per_poll: int = 2,
                 keep_displacements: bool = False, clock=time.perf_counter):
        self.engine = engine
        self.mesh_ids = {k: engine.add_mesh(m.X, m.tets, m.fixed) for k, m in meshes.items()}
        self.footprint = {k: int(engine.job_footprint(mid)) for k, mid in self.mesh_ids.items()}
        self.budget = int(hbm_budget)
        self.max_jobs = int(max_jobs)
        self.params = params
        self.rounds_per_poll = int(rounds_per_poll)
        self.keep_u = keep_displacements
        self.clock = clock
        self.queue: collections.deque[Request] = collections.deque()
        self.running: dict[int, tuple[Request, float]] = {}   # slot -> (request, admitted time)
        self.idle: dict[str, list[int]] = {k: [] for k in meshes}   # finished slots kept allocated
        self.slot_mesh: dict[int, str] = {}
        self.bytes_in_use = 0
        self.stats = ServerStats()
        self.results: list[Result] = []
        self.t0 = None

    # -- admission ---------------------------------------------------------
    def _live_slots(self) -> int:
        return len(self.slot_mesh)

    def _admit_one(self, req: Request, now: float) -> bool:
        key = req.mesh
        if self.idle[key]:
            slot = self.idle[key].pop()
            self.engine.restart_job(slot, req.indentation, req.E, req.nu)
            self.stats.restarted_in_place += 1
        else:
            fp = self.footprint[key]
            while (self.bytes_in_use + fp > self.budget or self._live_slots() >= self.max_jobs) and self._release_idle(key):
                pass
            if self.bytes_in_use + fp > self.budget or self._live_slots() >= self.max_jobs:
                self.stats.waits_for_memory += 1
                return False
            slot = self.engine.add_job(self.mesh_ids[key], req.indentation, req.E, req.nu)
            self.slot_mesh[slot] = key
            self.bytes_in_use += fp
            self.stats.allocated += 1
            self.stats.peak_bytes = max(self.stats.peak_bytes, self.bytes_in_use)
        self.running[slot] = (req, now)
        self.stats.admitted += 1
        self.stats.peak_running = max(self.stats.peak_running, len(self.running))
        return True

    def _release_idle(self, want: str) -> bool:
        """Frees one idle slot of a mesh other than `want`; False if none."""
        for key, slots in self.idle.items():
            if key != want and slots:
                slot = slots.pop()
                self.engine.remove_job(slot)
                self.bytes_in_use -= self.footprint[key]
                del self.slot_mesh[slot]
                self.stats.released += 1
                return True
        return False

    def _admit(self, now: float):
        while self.queue and self.queue[0].arrival <= now:
            req = self.queue[0]
            if self.footprint[req.mesh] > self.budget:
                # never admissible: refused with an error result, not queued forever
                self.queue.popleft()
                self.stats.rejected += 1
                self.results.append(Result(req.rid, req.mesh, req.arrival, now, now, REJECTED_FOOTPRINT, 0, 0, 0, 0))
                continue
            if not self._admit_one(req, now):
                if not self.running:
                    # with nothing running every idle slot could be released,
                    # so a request within the budget always fits
                    raise RuntimeError(f"request {req.rid} cannot be admitted with no job running")
                break
            self.queue.popleft()

    # -- completion ----------------------------------------------------------
    def _collect(self, now: float):
        for slot in list(self.running):
            info = self.engine.job_info(slot)
            if not info["done"]:
                continue
            req, admitted = self.running.pop(slot)
            u = self.engine.displacements(slot) if self.keep_u else None
            done = self.clock() - self.t0
            self.results.append(Result(req.rid, req.mesh, req.arrival, admitted, done, info["status"],
                                       info["steps_ok"], info["steps_failed"], info["cg_iters"],
                                       info["tet_updates"], u))
            self.idle[req.mesh].append(slot)

    # -- main loop -------------------------------------------------------------
    def serve(self, requests, timeout: float | None = None, progress=None, progress_every: float = 30.0):
        """Serves `requests` (sorted by arrival) until all are done; with
        `progress`, calls it with a status line every progress_every seconds."""
        self.queue.extend(sorted(requests, key=lambda r: r.arrival))
        total = len(self.queue)
        self.t0 = self.clock()
        next_report = progress_every
        while len(self.results) < total:
            now = self.clock() - self.t0
            if timeout is not None and now > timeout:
                raise TimeoutError(f"{len(self.results)} of {total} requests done after {now:.1f} s")
            if progress and now >= next_report:
                progress(f"serving: {len(self.results)} of {total} done at {now:.0f} s, {len(self.running)} running, "
                         f"{len(self.queue)} queued")
                next_report += progress_every
            self._admit(now)
            if not self.running:
                if self.queue:
                    wait = self.queue[0].arrival - (self.clock() - self.t0)
                    if wait > 0:
                        time.sleep(min(wait, 0.01))
                continue
            self.engine.run(self.params, max_rounds=self.rounds_per_poll)
            self.stats.rounds += self.rounds_per_poll
            self._collect(self.clock() - self.t0)
        return sorted(self.results, key=lambda r: r.rid)


def latency_summary(results, skip: int = 0) -> dict:
    """p50/p99/mean/max latency and solves/s of the served requests with rid
    >= skip (the first `skip` requests warm the server up): solves/s counts
    those requests over the span from the first one's arrival to the last
    completion."""
    results = [r for r in results if r.status != REJECTED_FOOTPRINT and r.rid >= skip]
    lat = np.array([r.latency for r in results]) * 1e3
    span = max(r.done for r in results) - min(r.arrival for r in results)
    return {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "max_ms": float(lat.max()), "completed": len(results),
            "solves_per_s": len(results) / span if span > 0 else float("nan"),
            "failed_load_steps": int(sum(r.steps_failed for r in results))}
