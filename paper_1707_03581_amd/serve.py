"""Continuous-batching request loop for look-ahead simulations on one GPU.

Requests (a machine at one of a few mesh levels, a horizon, and its own
Robin h, contact alpha, friction power, motion period and initial field)
arrive over time.  Each mesh level has one batched context (shared operators,
up to 64 slots) driven by its own host thread, so the levels' kernels run
concurrently on separate HIP streams.  A request is admitted into a free slot
of its level as soon as it has arrived and the level's context fits the HBM
budget; every scheduler tick advances all active slots of a level by one
macro-step (predictor + K sweeps); a request leaves when its horizon is done
and its slot is reused.  All arithmetic runs in libmrsdc.so; this module only
schedules and records latencies.
"""
from __future__ import annotations

import threading
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import BatchContext, config_from_scheme, load_problem


@dataclass
class Request:
    id: int
    arrival: float          # seconds after the start of the run
    level: str
    nsteps: int
    h: float
    alpha: float
    friction_W: float
    period: float
    T0: np.ndarray
    # filled by the server
    admitted: float = float("nan")
    finished: float = float("nan")
    step_ms: list = field(default_factory=list)
    result: np.ndarray = None
    slot: int = -1


def slot_bytes(pb) -> int:
    """Device bytes one scenario slot needs on a level (state vectors, caches)."""
    sc = pb.scheme
    n_if = 0
    c = pb.coupling
    if c is not None:
        F = pb.bodies[c.fix_body].faces[c.fix_face]
        G = pb.bodies[c.mov_body].faces[c.mov_face]
        n_if = F.nu * F.nv + G.nu * G.nv
    vectors = 3 * sc.M + 6
    return int(8 * pb.N * vectors + 16 * (sc.M + 1) * (sc.P + 1) * n_if)


class _Level:
    def __init__(self, name, pb, slots, device):
        self.name = name
        self.pb = pb
        self.slots = slots
        self.ctx = BatchContext(config_from_scheme(pb.scheme, device=device), slots)
        load_problem(self.ctx, pb, temperature=False)
        self.free = list(range(slots))
        self.active = {}  # slot -> Request
        for s in range(slots):
            self.ctx.set_active(s, False)
        self.ctx.advance_steps(0)  # build and upload the operators before serving


class Server:
    """levels: name -> problem description (shared mesh, scheme) of that level."""

    def __init__(self, levels: dict, slots_per_level: int = 64, hbm_budget_bytes: int = 200 << 30,
                 device: int = 0):
        self.levels_pb = levels
        self.slots = slots_per_level
        self.budget = hbm_budget_bytes
        self.device = device

    def run(self, requests: list, time_limit: float = 600.0):
        """Replay requests (sorted by arrival); returns them with timings and results."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        by_level = {name: [r for r in reqs if r.level == name] for name in self.levels_pb}
        levels = {}
        used = 0
        for name, pb in self.levels_pb.items():
            if not by_level[name]:
                continue
            slots = min(self.slots, len(by_level[name]))
            need = slots * slot_bytes(pb) + 40 * pb.nnz
            while slots > 1 and used + need > self.budget:
                slots //= 2
                need = slots * slot_bytes(pb) + 40 * pb.nnz
            if used + need > self.budget:
                raise MemoryError(f"level {name} does not fit the HBM budget")
            used += need
            levels[name] = _Level(name, pb, slots, self.device)
        self.footprint = {n: lv.ctx.footprint_bytes() for n, lv in levels.items()}
        t0 = time.perf_counter()
        errors = []

        def worker(lv: _Level, pending: list):
            try:
                todo = deque(pending)
                while todo or lv.active:
                    now = time.perf_counter() - t0
                    if now > time_limit:
                        raise TimeoutError(f"level {lv.name}: time limit")
                    # admit arrived requests into free slots
                    while todo and todo[0].arrival <= now and lv.free:
                        r = todo.popleft()
                        s = lv.free.pop()
                        lv.ctx.set_scenario(s, r.h, r.alpha, r.friction_W, r.period)
                        lv.ctx.set_scenario_temperature(s, r.T0)
                        lv.ctx.set_scenario_time(s, 0.0)
                        lv.ctx.set_active(s, True)
                        r.slot = s
                        r.admitted = time.perf_counter() - t0
                        lv.active[s] = r
                    if not lv.active:
                        wait = todo[0].arrival - (time.perf_counter() - t0) if todo else 0.0
                        time.sleep(min(max(wait, 0.0), 0.01))
                        continue
                    s0 = time.perf_counter()
                    lv.ctx.advance_steps(1)
                    ms = (time.perf_counter() - s0) * 1e3
                    for s, r in list(lv.active.items()):
                        r.step_ms.append(ms)
                        if len(r.step_ms) == r.nsteps:
                            r.result = lv.ctx.get_scenario_temperature(s, lv.pb.N)
                            r.finished = time.perf_counter() - t0
                            lv.ctx.set_active(s, False)
                            del lv.active[s]
                            lv.free.append(s)
            except BaseException as e:  # surfaced to the caller
                errors.append(e)

        threads = [threading.Thread(target=worker, args=(lv, by_level[n]), daemon=True)
                   for n, lv in levels.items()]
        for t in threads:
            t.start()
        for t in threads:
            t.join()
        self.wall = time.perf_counter() - t0
        for lv in levels.values():
            lv.ctx.destroy()
        if errors:
            raise errors[0]
        return reqs


def summarize(reqs, dt, dof_of_level):
    """Latency and throughput figures of a finished run."""
    lat = np.concatenate([np.asarray(r.step_ms) for r in reqs])
    wall = max(r.finished for r in reqs) - min(r.arrival for r in reqs)
    dof_steps = sum(dof_of_level[r.level] * r.nsteps for r in reqs)
    eta = [r.nsteps * dt / (r.finished - r.arrival) for r in reqs]
    eta_service = [r.nsteps * dt / (r.finished - r.admitted) for r in reqs]
    queue = [r.admitted - r.arrival for r in reqs]
    return {
        "requests": len(reqs),
        "p50_step_ms": float(np.percentile(lat, 50)),
        "p99_step_ms": float(np.percentile(lat, 99)),
        "dof_steps_per_s": dof_steps / wall,
        "wall_s": wall,
        "eta_p50": float(np.percentile(eta, 50)),
        "eta_min": float(np.min(eta)),
        "eta_service_p50": float(np.percentile(eta_service, 50)),
        "queue_p50_s": float(np.percentile(queue, 50)),
        "queue_max_s": float(np.max(queue)),
    }
