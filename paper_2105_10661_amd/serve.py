"""Continuous-batching driver for EMT contingency cases (host loop around serve_*).

Cases arrive over time (Poisson arrivals from ``cases.serve_arrivals``).  A
case is admitted when a slot is free and its device workspace fits the HBM
budget.  The workspace size comes from the library's host-only query
(``emt_workspace_size``) before anything is built, so a case that waits for
memory costs nothing on the device; a case larger than the whole budget is
refused and reported, never admitted.  Admitted cases are built (hierarchy,
SMW factors) and attached to the pool; every tick is one launch that advances
all attached cases by ``tick_steps`` steps; a case whose steps are done is
detached and its memory released, which admits waiting cases.  Times are
wall-clock on the host with the stream synchronised at every tick.

The budget counts the workspaces the library asks for; the caching allocator
of torch may hold more than that (freed blocks are kept for reuse).
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np


@dataclass
class ServeResult:
    completed: int = 0
    solves: int = 0
    wall_s: float = 0.0
    tick_us: List[float] = field(default_factory=list)       # per-step latency of each tick (tick time / steps)
    max_active: int = 0
    queue_wait_s: List[float] = field(default_factory=list)
    refused: List[int] = field(default_factory=list)        # arrivals larger than the whole budget
    created: int = 0                                          # EMT contexts built (one per admitted case)
    records: Dict[int, np.ndarray] = field(default_factory=dict)

    @property
    def solves_per_s(self) -> float:
        return self.solves / self.wall_s if self.wall_s > 0 else 0.0


def run_serving(arrivals, budget_bytes: int, max_slots: int = 256, tick_steps: int = 100, prec: str = "fp32",
                warm_start: bool = True, max_refine: int = 2, rel_tol: float = 1e-9, record: bool = False,
                time_scale: float = 1.0, max_wall_s: Optional[float] = None, pool=None) -> ServeResult:
    """Serve `arrivals` (list of cases.Arrival); returns throughput and latency statistics.

    record=True keeps every case's full trajectory (for checks; costs memory).
    time_scale stretches the arrival clock (1.0 = real time; 0 = everything has arrived).
    pool: a ``hinv.Serve`` (default: a new one with these settings, closed at the end).
    """
    from . import hinv

    own = pool is None
    if own:
        pool = hinv.Serve(max_slots, prec=prec, warm_start=warm_start, max_refine=max_refine, rel_tol=rel_tol)
    res = ServeResult()
    pending = sorted(range(len(arrivals)), key=lambda i: arrivals[i].t)
    active = {}          # slot -> (index, emt, remaining steps, record, bytes)
    used = 0
    need = {}            # arrival index -> workspace bytes
    t0 = time.perf_counter()
    while pending or active:
        now = (time.perf_counter() - t0) / time_scale if time_scale > 0 else float("inf")
        # admission: arrived cases in arrival order while a slot and budget are free
        while pending and arrivals[pending[0]].t <= now and len(active) < max_slots:
            i = pending[0]
            case = arrivals[i].case
            losses = list(zip(case.loss_steps.tolist(), case.loss_branches.tolist()))
            if i not in need:          # host-only size query: nothing is built for a case that waits
                need[i] = pool.case_bytes(case.net, losses, max_mod_rank=max(1, len(losses)))
            if need[i] > budget_bytes:
                pending.pop(0)
                res.refused.append(i)
                continue
            if used + need[i] > budget_bytes:
                break
            pending.pop(0)
            emt = pool.new_case(case.net, losses, max_mod_rank=max(1, len(losses)))
            res.created += 1
            sid, rec = pool.attach(emt, record_steps=case.n_steps if record else 0)
            active[sid] = (i, emt, case.n_steps, rec, need[i])
            used += need[i]
            res.queue_wait_s.append(max(0.0, now - arrivals[i].t))
        res.max_active = max(res.max_active, len(active))
        if not active:
            if not pending:
                break
            time.sleep(max(0.0, min(0.001, arrivals[pending[0]].t * time_scale - (time.perf_counter() - t0))))
            continue
        k = min(tick_steps, min(a[2] for a in active.values()))
        ts = time.perf_counter()
        pool.step(k)
        pool.synchronize()
        res.tick_us.append((time.perf_counter() - ts) / k * 1e6)
        res.solves += k * len(active)
        done = []
        for sid, (i, emt, rem, rec, nb) in active.items():
            if rem - k <= 0:
                done.append(sid)
            else:
                active[sid] = (i, emt, rem - k, rec, nb)
        for sid in done:
            i, emt, rem, rec, nb = active.pop(sid)
            pool.detach(sid)
            if rec is not None:
                res.records[i] = rec.cpu().numpy()
            emt.close()
            used -= nb
            res.completed += 1
        if max_wall_s is not None and time.perf_counter() - t0 > max_wall_s:
            break
    res.wall_s = time.perf_counter() - t0
    for sid, (i, emt, rem, rec, nb) in active.items():     # stopped early (max_wall_s)
        pool.detach(sid)
        emt.close()
    if own:
        pool.close()
    return res
