"""Continuous-batching request loop for look-ahead simulations on one GPU.

Requests (a machine at one of a few mesh levels, a horizon, and its own
Robin h, contact alpha, friction power, motion period and initial field)
arrive over time.  Each mesh level has one batched context (shared operators,
a pool of scenario slots whose node states stay resident on the device)
driven by its own host thread, so the levels' kernels run concurrently on
separate HIP streams.

Admission by HBM footprint: before the replay, each configured level's
footprint is taken from the library (bytes shared by the level, bytes per
scenario slot) and the levels' slot pools are sized so that their device
memory together stays within the HBM budget (default: 90 % of the device
memory free at start).  A level that cannot hold its operators and one slot
within what is left gets no pool, and its requests are rejected on arrival.
A request of a pooled level is admitted into a free slot as soon as it has
arrived; while every slot is taken it waits in its level's queue.  Every
scheduler tick advances all active slots of a level by one macro-step
(predictor + K sweeps); a request leaves when its horizon is done and its slot
is reused.  All arithmetic runs in libmrsdc.so; this module only schedules,
accounts memory and records latencies.
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
    rejected: bool = False
    step_ms: list = field(default_factory=list)
    result: np.ndarray = None
    slot: int = -1


def plan_pools(level_bytes: dict, budget: int, slots_per_level: int) -> dict:
    """Slots per level within an HBM budget.

    level_bytes: name -> (shared bytes, bytes per slot) as the library reports
    them.  Levels are served in order of their one-slot footprint (smallest
    first), each taking up to slots_per_level slots of what is left of the
    budget; a level that cannot hold its shared bytes and one slot gets 0
    (its requests are rejected).  The order and the sizes depend only on the
    configured levels, never on the requests to come."""
    plan = {}
    left = int(budget)
    for name in sorted(level_bytes, key=lambda n: sum(level_bytes[n])):
        shared, per = level_bytes[name]
        fit = (left - shared) // per if left >= shared + per else 0
        slots = int(min(slots_per_level, fit))
        plan[name] = slots
        if slots:
            left -= shared + slots * per
    return plan


def level_bytes(pb, device=0):
    """(shared, per-slot) device bytes of a level, from a one-slot context."""
    ctx = BatchContext(config_from_scheme(pb.scheme, device=device), 1)
    try:
        load_problem(ctx, pb, temperature=False)
        ctx.set_active(0, False)
        ctx.advance_steps(0)  # builds the device state
        per, shared = ctx.slot_bytes()
    finally:
        ctx.destroy()
    return shared, per


def default_budget(device=0) -> int:
    import torch
    free, _ = torch.cuda.mem_get_info(device)
    return int(0.9 * free)


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
    """levels: name -> problem description (shared mesh, scheme) of that level.
    hbm_budget_bytes: device memory the pools may hold (None: 90 % of the
    device memory free when run() starts)."""

    def __init__(self, levels: dict, slots_per_level: int = 64, hbm_budget_bytes=None,
                 device: int = 0):
        self.levels_pb = levels
        self.slots = slots_per_level
        self.budget = hbm_budget_bytes
        self.device = device

    def size_pools(self):
        """Footprints from the library and the slot plan within the budget."""
        if self.budget is None:
            self.budget = default_budget(self.device)
        self.level_bytes = {n: level_bytes(pb, self.device) for n, pb in self.levels_pb.items()}
        self.plan = plan_pools(self.level_bytes, self.budget, self.slots)
        return self.plan

    def run(self, requests: list, time_limit: float = 600.0):
        """Replay requests (sorted by arrival); returns them with timings and
        results (rejected requests keep result None)."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        if not hasattr(self, "plan"):
            self.size_pools()
        levels = {}
        for name, slots in self.plan.items():
            if slots:
                levels[name] = _Level(name, self.levels_pb[name], slots, self.device)
        self.footprint = {n: lv.ctx.footprint_bytes() for n, lv in levels.items()}
        self.held_bytes = sum(self.footprint.values())
        if self.held_bytes > self.budget:
            for lv in levels.values():
                lv.ctx.destroy()
            raise MemoryError(f"pools hold {self.held_bytes} bytes, budget {self.budget}")
        by_level = {name: [r for r in reqs if r.level == name] for name in levels}
        for r in reqs:
            if r.level not in levels:
                r.rejected = True
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
    """Latency and throughput figures of a finished run (served requests;
    rejected ones are counted apart)."""
    served = [r for r in reqs if not r.rejected]
    out = {"requests": len(reqs), "served": len(served), "rejected": len(reqs) - len(served)}
    if not served:
        return out
    lat = np.concatenate([np.asarray(r.step_ms) for r in served])
    wall = max(r.finished for r in served) - min(r.arrival for r in served)
    dof_steps = sum(dof_of_level[r.level] * r.nsteps for r in served)
    eta = [r.nsteps * dt / (r.finished - r.arrival) for r in served]
    eta_service = [r.nsteps * dt / (r.finished - r.admitted) for r in served]
    queue = [r.admitted - r.arrival for r in served]
    out.update({
        "p50_step_ms": float(np.percentile(lat, 50)),
        "p99_step_ms": float(np.percentile(lat, 99)),
        "dof_steps_per_s": dof_steps / wall,
        "wall_s": wall,
        "eta_p50": float(np.percentile(eta, 50)),
        "eta_min": float(np.min(eta)),
        "eta_service_p50": float(np.percentile(eta_service, 50)),
        "queue_p50_s": float(np.percentile(queue, 50)),
        "queue_max_s": float(np.max(queue)),
    })
    return out
