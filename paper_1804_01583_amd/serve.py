"""Serving loop: a stream of verification queries on one GPU.

Queries arrive over time (each a set of box generators, output rows, an
unsafe threshold, a time grid and a precision against one of the resident
systems).  The server

* admits a waiting query as soon as a slot is free and the HBM budget
  covers its plan's workspace (kry_plan_workspace): the oldest one, or,
  when the oldest does not fit, the oldest one behind it that does; a query
  passed over `max_bypass` times is then waited for (the others stay queued
  until it fits), so a large query delays later small ones by a bounded
  amount instead of stalling the queue,
* batches an admitted query with the waiting queries on the same resident
  system, precision, time step and Krylov dimension (up to 8 output rows
  and 64 basis columns together): they become one plan whose runs are all
  their generators, so every mat-vec launch advances the same Krylov step
  of all of them, and each query's verdict is the box check over its own
  columns, rows and steps (kry_check_box_subset),
* runs admitted batches concurrently, each on its own HIP stream, so their
  kernels overlap on the device,
* keeps every plan's basis and state on the device until its verdict is
  read, and records arrival -> verdict latency.

A query's result does not depend on what runs beside it on other streams:
every kernel's arithmetic and reduction order depend only on its plan's
sizes.  In a batch, a run's Krylov data are those of the run alone (runs do
not interact); the longer time grid and the extra output rows of the batch's
plan change its per-step exponentials by rounding only.

Systems are resident: a catalog holds one device copy per (family, grid),
with the prepared matrix (sliced-ELL copy and norm) of each precision a
CSR system is queried in, and queries borrow them.
"""
from __future__ import annotations

import threading
import time
from collections import deque
from dataclasses import dataclass
from typing import Dict, List, Optional, Tuple

import numpy as np

from . import kry


class Catalog:
    """Device-resident systems keyed by (family, m), built on first use."""

    def __init__(self, device="cuda"):
        self.device = device
        self._systems: Dict[Tuple[str, int], "kry.DeviceSystem"] = {}
        self._lock = threading.Lock()

    def get(self, family: str, m: int, precision=None):
        """The resident system; with `precision`, a CSR system also holds its
        prepared matrix (sliced-ELL copy and norm) for that precision."""
        import workloads as W
        key = (family, m)
        with self._lock:
            if key not in self._systems:
                self._systems[key] = kry.DeviceSystem(W.serving_system(family, m), device=self.device)
            ds = self._systems[key]
            if precision is not None and ds.problem.kind == "csr":
                ds.prepare(precision)
            return ds

    def preload(self, queries):
        import torch
        for q in queries:
            self.get(q.family, q.m, _precision(q))
        torch.cuda.synchronize(self.device)

    def resident_bytes(self) -> int:
        total = 0
        for ds in self._systems.values():
            for name in ("rowptr", "colidx", "vals", "b", "center"):
                t = getattr(ds, name, None)
                if t is not None:
                    total += t.numel() * t.element_size()
            total += sum(kry.kry_matrix_bytes(h) for h in ds.prepared.values())
        return total


def _precision(q):
    return kry.KRY_FP32_BASIS if q.precision == "fp32" else kry.KRY_FP64


@dataclass
class Result:
    qid: int
    arrival: float
    admitted: float
    done: float
    verdict: dict
    footprint: int
    verified_steps: int
    basis: Optional[np.ndarray] = None
    group: int = 1            # queries in the plan that ran it
    cancelled: bool = False   # withdrawn by Server.cancel: verdict is {"cancelled": True}

    @property
    def latency(self) -> float:
        return self.done - self.arrival


@dataclass
class _Pending:
    query: object
    footprint: int
    released: float
    bypassed: int = 0


MAX_GROUP_ROWS = 8        # output rows of one plan
MAX_GROUP_COLS = 64       # basis columns one subset check takes


def group_key(q):
    """Queries that can share one plan: same resident system, precision,
    time step and Krylov dimension."""
    return (q.family, q.m, q.precision, q.dt, q.k)


def form_group(pending, first: int, max_queries: int = 8, fits=None):
    """Removes pending[first] and the later waiting queries with its key
    (oldest first) from `pending` and returns them: together at most
    MAX_GROUP_ROWS output rows, MAX_GROUP_COLS generators and max_queries
    queries; `fits(group)` may veto each addition (the HBM budget)."""
    head = pending[first]
    del pending[first]
    group = [head]
    key = group_key(head.query)
    rows, cols = len(head.query.C), len(head.query.gens)
    i = 0
    while i < len(pending) and len(group) < max_queries:
        q = pending[i].query
        if (group_key(q) == key and rows + len(q.C) <= MAX_GROUP_ROWS and cols + len(q.gens) <= MAX_GROUP_COLS
                and (fits is None or fits(group + [pending[i]]))):
            group.append(pending[i])
            rows += len(q.C)
            cols += len(q.gens)
            del pending[i]
        else:
            i += 1
    return group


def pick_admission(pending, in_use: int, budget: int, max_bypass: int, scan: int = 64):
    """Index into `pending` (oldest first) of the query to admit now, or None.
    The oldest query goes first when it fits (or when nothing runs: a query
    larger than the budget then runs alone).  Otherwise the oldest of the
    next `scan` queries that fits passes it, until the oldest has been passed
    `max_bypass` times; from then on it is waited for."""
    if not pending:
        return None
    head = pending[0]
    if in_use + head.footprint <= budget or in_use == 0:
        return 0
    if head.bypassed >= max_bypass:
        return None
    for i in range(1, min(len(pending), scan + 1)):
        if in_use + pending[i].footprint <= budget:
            head.bypassed += 1
            return i
    return None


class Server:
    """slots: queries in flight at once; budget_bytes: HBM for their plans.
    ``runner(query, slot, keep_basis) -> (verdict, basis, runs)`` and
    ``footprint(query) -> bytes`` default to the GPU plan and kry_plan_workspace;
    other ones serve for testing the scheduling on the host."""

    def __init__(self, catalog: Optional[Catalog], slots: int = 8, budget_bytes: int = 200 << 30,
                 runner=None, footprint=None, max_bypass: int = 16, batch: bool = True, max_group: int = 8):
        self.catalog = catalog
        self.slots = slots
        self.budget = budget_bytes
        self.max_bypass = max_bypass
        # batches need the GPU runner (a stand-in runner takes one query)
        self.max_group = max_group if (batch and runner is None) else 1
        self._runner = runner
        self._footprint = footprint
        self._cancel_lock = threading.Lock()
        self._cancelled = set()
        self._cond = None

    def cancel(self, qid: int) -> None:
        """Withdraws query qid (callable from any thread while serve runs).
        A query still waiting, or not yet arrived, never runs; one already
        running finishes on the device (its launches are not interrupted) and
        its verdict is dropped.  Either way its Result has cancelled=True and
        its slot and HBM are released as usual."""
        with self._cancel_lock:
            self._cancelled.add(qid)
            cond = self._cond
        if cond is not None:
            with cond:
                cond.notify_all()

    def _is_cancelled(self, qid: int) -> bool:
        with self._cancel_lock:
            return qid in self._cancelled

    def footprint(self, q) -> int:
        if self._footprint is not None:
            return self._footprint(q)
        prec = _precision(q)
        dsys = self.catalog.get(q.family, q.m, prec)
        nseg = sum(g.seg.nseg for g in q.gens) + sum(c.nseg for c in q.C)
        return kry.kry_plan_workspace(dsys.system_for(prec), len(q.gens), len(q.C), q.k, q.steps, nseg, prec,
                                 kry.KRY_AUTO, 0)

    def group_footprint(self, group) -> int:
        """Workspace of the plan that runs a group of _Pending queries."""
        if len(group) == 1:
            return group[0].footprint
        qs = [g.query for g in group]
        prec = _precision(qs[0])
        dsys = self.catalog.get(qs[0].family, qs[0].m, prec)
        nseg = sum(g.seg.nseg for q in qs for g in q.gens) + sum(c.nseg for q in qs for c in q.C)
        return kry.kry_plan_workspace(dsys.system_for(prec), sum(len(q.gens) for q in qs),
                                      sum(len(q.C) for q in qs), qs[0].k, max(q.steps for q in qs), nseg, prec,
                                      kry.KRY_AUTO, 0)

    def _run_group(self, qs, stream, keep_basis: bool):
        """One plan for all queries of a group: their generators are its
        runs, their output rows its rows, the longest time grid its steps;
        each query's verdict is the box check over its own columns, rows and
        steps.  Returns [(verdict, basis, columns)] in group order."""
        import torch
        prec = _precision(qs[0])
        dsys = self.catalog.get(qs[0].family, qs[0].m, prec)
        gens = [g for q in qs for g in q.gens]
        rows = [c for q in qs for c in q.C]
        steps = max(q.steps for q in qs)
        out_list = []
        with torch.cuda.stream(stream):
            plan = kry.Plan(dsys, k=qs[0].k, dt=qs[0].dt, steps=steps, precision=prec, stream=stream, gens=gens,
                            C=rows)
            out = None
            if keep_basis:
                out = torch.empty((steps + 1, len(rows), plan.nruns), dtype=torch.float64, device=dsys.device)
            plan.project_expm(out)
            c0 = r0 = 0
            for q in qs:
                g, o = len(q.gens), len(q.C)
                v, z = kry.kry_check_box_subset(plan.handle, np.arange(c0, c0 + g), np.arange(r0, r0 + o), q.steps,
                                                np.asarray(q.unsafe, np.float64), g)
                verdict = {"first_step": int(v.first_step), "row": int(v.row), "status": int(v.status), "y": v.y,
                           "lo": v.lo, "hi": v.hi, "z": z}
                basis = out[:q.steps + 1, r0:r0 + o, c0:c0 + g].cpu().numpy() if keep_basis else None
                out_list.append((verdict, basis, g))
                c0 += g
                r0 += o
            plan.close()
        return out_list

    def _run_one(self, q, stream, keep_basis: bool):
        import torch
        prec = _precision(q)
        dsys = self.catalog.get(q.family, q.m, prec)
        with torch.cuda.stream(stream):
            plan = kry.Plan(dsys, k=q.k, dt=q.dt, steps=q.steps, precision=prec, stream=stream, gens=q.gens, C=q.C)
            out = None
            if keep_basis:
                out = torch.empty((q.steps + 1, len(q.C), plan.nruns), dtype=torch.float64, device=dsys.device)
            plan.project_expm(out)
            verdict = plan.check(q.unsafe)          # waits for this stream only
            basis = out.cpu().numpy() if keep_basis else None
            runs = plan.nruns
            plan.close()
        return verdict, basis, runs

    def serve(self, queries, keep_basis: bool = False, time_scale: float = 1.0) -> List[Result]:
        """Plays the queries at their arrival times (times time_scale) and
        returns one Result per query, in query order."""
        order = sorted(queries, key=lambda q: q.arrival)
        pending: deque = deque()
        results: Dict[int, Result] = {}
        errors: List[BaseException] = []
        cond = threading.Condition()
        with self._cancel_lock:
            self._cond = cond
        state = {"in_use": 0, "dispatched": False}
        if self._runner is None:
            import torch
            streams = [torch.cuda.Stream(device=self.catalog.device) for _ in range(self.slots)]

            def run_group(qs, slot, keep):
                if len(qs) == 1:
                    return [self._run_one(qs[0], streams[slot], keep)]
                return self._run_group(qs, streams[slot], keep)
        else:
            def run_group(qs, slot, keep):
                return [self._runner(q, slot, keep) for q in qs]
        t0 = time.perf_counter()

        def drop(q, fp, admitted):
            # caller holds cond
            now = time.perf_counter() - t0
            results[q.qid] = Result(q.qid, q.arrival * time_scale, admitted if admitted is not None else now, now,
                                    {"cancelled": True}, fp, 0, None, 1, cancelled=True)

        def dispatcher():
            try:
                for q in order:
                    if errors:
                        break
                    fp = self.footprint(q)
                    wait = t0 + q.arrival * time_scale - time.perf_counter()
                    if wait > 0:
                        time.sleep(wait)
                    with cond:
                        if self._is_cancelled(q.qid):
                            drop(q, fp, None)
                        else:
                            pending.append(_Pending(q, fp, time.perf_counter() - t0))
                        cond.notify_all()
            finally:
                with cond:
                    state["dispatched"] = True
                    cond.notify_all()

        def worker(slot):
            while True:
                with cond:
                    while True:
                        if errors:
                            return
                        for item in [p for p in pending if self._is_cancelled(p.query.qid)]:
                            pending.remove(item)
                            drop(item.query, item.footprint, None)
                        i = pick_admission(pending, state["in_use"], self.budget, self.max_bypass)
                        if i is not None:
                            in_use = state["in_use"]
                            group = form_group(
                                pending, i, self.max_group,
                                fits=lambda g: in_use + self.group_footprint(g) <= self.budget)
                            fp = self.group_footprint(group)
                            state["in_use"] += fp
                            break
                        if state["dispatched"] and not pending:
                            return
                        cond.wait()
                admitted = time.perf_counter() - t0
                try:
                    outs = run_group([g.query for g in group], slot, keep_basis)
                except BaseException as e:  # noqa: BLE001 - surfaced after the threads stop
                    with cond:
                        errors.append(e)
                        state["in_use"] -= fp
                        cond.notify_all()
                    return
                done = time.perf_counter() - t0
                with cond:
                    state["in_use"] -= fp
                    for item, (verdict, basis, runs) in zip(group, outs):
                        q = item.query
                        if self._is_cancelled(q.qid):
                            drop(q, fp, admitted)
                            continue
                        results[q.qid] = Result(q.qid, q.arrival * time_scale, admitted, done, verdict, fp,
                                                (q.steps + 1) * runs, basis, len(group))
                    cond.notify_all()

        threads = [threading.Thread(target=worker, args=(s,), daemon=True) for s in range(self.slots)]
        for t in threads:
            t.start()
        dispatcher()
        for t in threads:
            t.join()
        with self._cancel_lock:
            self._cond = None
        if errors:
            raise errors[0]
        return [results[q.qid] for q in queries]


def summarize(results: List[Result]) -> dict:
    """Latency and throughput over the queries that were not cancelled."""
    cancelled = sum(r.cancelled for r in results)
    results = [r for r in results if not r.cancelled]
    lat = np.array([r.latency for r in results])
    span = max(r.done for r in results) - min(r.arrival for r in results)
    steps = sum(r.verified_steps for r in results)
    return {"queries": len(results), "cancelled": cancelled, "p50_ms": 1000.0 * float(np.percentile(lat, 50)),
            "p99_ms": 1000.0 * float(np.percentile(lat, 99)), "max_ms": 1000.0 * float(lat.max()),
            "verified_steps_per_s": steps / span if span > 0 else float("nan"), "span_s": span,
            "unsafe": int(sum(r.verdict["first_step"] >= 0 for r in results)),
            "mean_group": float(np.mean([r.group for r in results]))}
