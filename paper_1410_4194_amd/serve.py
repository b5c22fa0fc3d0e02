"""Continuous-batching request loop for independent CTU solves (the serving form).

Requests arrive over time; each carries its initial state (a :class:`Workload`), an end
time and a precision.  The loop admits requests in arrival order while their device
footprint (state + workspace) fits an HBM budget and a batch slot is free, advances every
admitted grid together (one launch per pass over all running grids, ``ctu.Batch``, each grid
with its own device-side time step), and retires a grid when it reaches its end time:
its solution is downloaded and its memory released, which may admit the next request.
Requests that arrive while others run join the running set at the next round, so their
work overlaps on the device.

Two admission policies: "fifo" admits in arrival order and stops at the first arrived
request that does not fit (no request overtakes an earlier one); "sjf" admits, among the
requests that have arrived, the one with the least estimated work (``Request.cost``, the
caller's estimate, e.g. cells x estimated steps) that fits, so small requests do not wait
behind a large one for memory.

Time-to-solution of a request is measured from its arrival to its solution on the host.
All arithmetic runs in the library's kernels; this module only schedules.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional

import numpy as np

from . import ctu


@dataclass
class Request:
    rid: int
    arrival: float            # seconds after the loop starts
    workload: object          # workloads.Workload: geometry, gamma, boundaries, initial state
    t_end: float
    prec: int = ctu.FP32
    max_steps: int = 1 << 30
    cost: float = 0.0          # estimated work (any unit), for the "sjf" admission policy


@dataclass
class Result:
    rid: int
    arrival: float
    admitted: float
    finished: float
    steps: int
    t: float
    cells: int
    state: Optional[np.ndarray] = None

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


@dataclass
class ServeStats:
    results: List[Result]
    makespan: float
    max_resident_bytes: int
    max_concurrent: int
    rounds: int
    extra: Dict[str, float] = field(default_factory=dict)

    def summary(self) -> dict:
        lat = np.array([r.latency for r in self.results])
        work = sum(r.cells * r.steps for r in self.results)
        wait = np.array([r.admitted - r.arrival for r in self.results])
        return {"requests": len(self.results),
                "p50_s": round(float(np.percentile(lat, 50)), 4),
                "p99_s": round(float(np.percentile(lat, 99)), 4),
                "mean_s": round(float(lat.mean()), 4),
                "mean_admission_wait_s": round(float(wait.mean()), 4),
                "cell_updates": int(work),
                "cell_updates_per_s": round(work / self.makespan, 1),
                "makespan_s": round(self.makespan, 3),
                "max_resident_gb": round(self.max_resident_bytes / 1e9, 3),
                "max_concurrent": self.max_concurrent, "rounds": self.rounds}


def footprint(req: Request) -> int:
    wl = req.workload
    cfg = ctu.make_config(wl.nx, wl.ny, wl.nz, wl.dx, wl.dy, wl.dz, wl.gamma, wl.bc, req.prec,
                          wl.cfl)
    sb, wb = ctu.workspace_bytes(cfg)
    return sb + wb


POLICIES = ("fifo", "sjf")


def next_admission(pending: List[Request], now: float, free_bytes: int, free_slots: int,
                   need: Callable[[Request], int], policy: str = "fifo") -> Optional[int]:
    """Index into `pending` (sorted by arrival) of the request to admit next, or None.
    fifo: the earliest arrival, if it fits; sjf: the least `cost` among the arrived requests
    that fit (ties by arrival)."""
    if free_slots <= 0:
        return None
    if policy == "fifo":
        if pending and pending[0].arrival <= now and need(pending[0]) <= free_bytes:
            return 0
        return None
    if policy != "sjf":
        raise ValueError(f"unknown admission policy {policy!r}")
    best = None
    for i, r in enumerate(pending):
        if r.arrival > now:
            break
        if need(r) <= free_bytes and (best is None or r.cost < pending[best].cost):
            best = i
    return best


def serve(requests: List[Request], hbm_budget: int, max_slots: int = 64,
          steps_per_round: int = 8, graph: bool = True, keep_states: bool = False,
          clock: Callable[[], float] = time.perf_counter, policy: str = "fifo") -> ServeStats:
    """Run the request loop until every request is answered.

    Each round enqueues `steps_per_round` steps of the running grids first; while the GPU
    works, the host downloads the solutions retired in the previous round and admits new
    arrivals (uploads go through a stream of their own, so they overlap the round); then one
    poll (a single read-back for all slots) finds the grids that are done."""
    import torch

    if policy not in POLICIES:
        raise ValueError(f"unknown admission policy {policy!r}")
    pending = sorted(requests, key=lambda r: (r.arrival, r.rid))
    need_of = {r.rid: footprint(r) for r in pending}
    for r in pending:
        if need_of[r.rid] > hbm_budget:
            raise ValueError(f"request {r.rid} needs more than the HBM budget")
    io_stream = torch.cuda.Stream()
    batch = ctu.Batch(max_slots, graph=graph)
    active = {}   # ticket -> (request, grid, admitted time, bytes)
    retire = []   # (request, grid, admitted time, bytes, t) found done by the last poll
    results = []
    resident = 0
    max_resident = 0
    max_conc = 0
    rounds = 0
    t0 = clock()
    try:
        while pending or active or retire:
            if active:
                batch.run(steps_per_round)
                rounds += 1
            # host work overlapping the round: hand back finished solutions ...
            for req, g, admitted, need, t_now in retire:
                U = g.get_state()
                steps = g.info().steps
                wl = req.workload
                results.append(Result(req.rid, req.arrival, admitted, clock() - t0, steps,
                                      t_now, wl.nx * wl.ny * wl.nz, U if keep_states else None))
                g.close()
                resident -= need
            retire = []
            # ... and admit arrivals (by the policy) while memory and slots allow
            now = clock() - t0
            while True:
                i = next_admission(pending, now, hbm_budget - resident, max_slots - len(active),
                                   lambda r: need_of[r.rid], policy)
                if i is None:
                    break
                req = pending[i]
                need = need_of[req.rid]
                g = ctu.Grid.from_workload(req.workload, prec=req.prec, stream=io_stream,
                                           batch=True)
                ticket = batch.submit(g, req.max_steps, req.t_end)
                if ticket is None:
                    g.close()
                    break
                del pending[i]
                resident += need
                active[ticket] = (req, g, clock() - t0, need)
                now = clock() - t0
            max_resident = max(max_resident, resident)
            max_conc = max(max_conc, len(active))
            if not active:
                if pending and not retire:
                    time.sleep(max(0.0, pending[0].arrival - (clock() - t0)))
                continue
            for ticket in list(active):
                state, t_now = batch.poll(ticket)
                if state == ctu.TICKET_RUNNING:
                    continue
                req, g, admitted, need = active.pop(ticket)
                if state != ctu.TICKET_DONE:
                    raise RuntimeError(f"request {req.rid} failed (non-physical state)")
                retire.append((req, g, admitted, need, t_now))
        first = min(r.arrival for r in requests) if requests else 0.0
        makespan = clock() - t0 - first
    finally:
        batch.close()
    results.sort(key=lambda r: r.rid)
    return ServeStats(results, makespan, max_resident, max_conc, rounds)
