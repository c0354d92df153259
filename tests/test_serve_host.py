"""Scheduling of the serving loop on the host (no GPU): arrival order,
admission by the HBM budget and by free slots, latency accounting, error
propagation.  The runner is a stand-in that sleeps; the GPU runner is
exercised by tests/test_gpu_serve.py."""
import threading
import time

import numpy as np
import pytest

import workloads as W
from paper_1804_01583_amd.serve import Server, summarize


def _fake(service_s, log, lock):
    def run(q, slot, keep):
        with lock:
            log.append(("start", q.qid, time.perf_counter()))
        time.sleep(service_s)
        with lock:
            log.append(("end", q.qid, time.perf_counter()))
        return {"first_step": -1, "row": -1}, None, len(q.gens)
    return run


def test_fifo_admission_and_budget():
    qs = W.serving_queries(24, rate=200.0, seed=300)
    fp = {q.qid: 10 + (q.qid % 3) * 10 for q in qs}       # 10, 20 or 30 units
    log, lock = [], threading.Lock()
    # max_bypass=0: strict arrival order
    srv = Server(None, slots=4, budget_bytes=45, runner=_fake(0.02, log, lock), footprint=lambda q: fp[q.qid],
                 max_bypass=0)
    res = srv.serve(qs)
    # admission is in arrival order
    starts = [e[1] for e in log if e[0] == "start"]
    assert starts == sorted(starts, key=lambda i: qs[i].arrival)
    # at no time do the running queries exceed the budget or the slots
    events = sorted(log, key=lambda e: (e[2], e[0] == "start"))
    running = set()
    for kind, qid, _ in events:
        if kind == "start":
            running.add(qid)
            assert len(running) <= 4
            assert sum(fp[i] for i in running) <= 45
        else:
            running.discard(qid)
    # latency = done - arrival >= the service time, admission after arrival
    for r in res:
        assert r.admitted >= r.arrival - 1e-3
        assert r.latency >= 0.02 - 1e-3
    s = summarize(res)
    assert s["queries"] == 24 and s["p99_ms"] >= s["p50_ms"] > 0


def test_small_queries_pass_a_blocked_head_a_bounded_number_of_times():
    # the third query needs 40 of 50 units: while two 20-unit queries run it
    # does not fit, and later small queries go first, at most max_bypass of
    # them; the budget and the slots hold throughout
    qs = W.serving_queries(30, rate=2000.0, seed=303)
    big = qs[2].qid
    fp = {q.qid: (40 if q.qid == big else 20) for q in qs}
    log, lock = [], threading.Lock()
    srv = Server(None, slots=4, budget_bytes=50, runner=_fake(0.01, log, lock), footprint=lambda q: fp[q.qid],
                 max_bypass=3)
    srv.serve(qs)
    starts = [e[1] for e in log if e[0] == "start"]
    pos = starts.index(big)
    later = [i for i in starts[:pos] if qs[i].arrival > qs[big].arrival]
    assert 1 <= len(later) <= 3, starts
    events = sorted(log, key=lambda e: (e[2], e[0] == "start"))
    running = set()
    for kind, qid, _ in events:
        if kind == "start":
            running.add(qid)
            assert len(running) <= 4 and sum(fp[i] for i in running) <= 50
        else:
            running.discard(qid)


def test_pick_admission_rules():
    from paper_1804_01583_amd.serve import _Pending, pick_admission
    P = [_Pending(None, f, 0.0) for f in (40, 10, 30, 5)]
    assert pick_admission(P, 0, 50, 2) == 0            # nothing running: the oldest, whatever its size
    assert pick_admission(P, 20, 50, 2) == 1           # 40 does not fit beside 20: the 10 goes first
    assert P[0].bypassed == 1
    assert pick_admission(P, 20, 50, 2) == 1
    assert pick_admission(P, 20, 50, 2) is None        # passed twice: now it is waited for
    assert pick_admission(P, 10, 50, 2) == 0
    assert pick_admission([], 0, 50, 2) is None


def test_oversized_query_runs_alone():
    qs = W.serving_queries(5, rate=1000.0, seed=301)
    log, lock = [], threading.Lock()
    big = qs[2].qid
    srv = Server(None, slots=3, budget_bytes=100, runner=_fake(0.01, log, lock),
                 footprint=lambda q: 500 if q.qid == big else 10)
    srv.serve(qs)
    t_start = {e[1]: e[2] for e in log if e[0] == "start"}
    t_end = {e[1]: e[2] for e in log if e[0] == "end"}
    for q in qs:
        if q.qid != big:
            overlap = t_start[q.qid] < t_end[big] and t_start[big] < t_end[q.qid]
            assert not overlap


def test_runner_error_is_raised():
    qs = W.serving_queries(6, rate=1000.0, seed=302)

    def run(q, slot, keep):
        if q.qid == 3:
            raise RuntimeError("query 3 failed")
        return {"first_step": -1, "row": -1}, None, 1
    srv = Server(None, slots=2, budget_bytes=1 << 40, runner=run, footprint=lambda q: 1)
    with pytest.raises(RuntimeError, match="query 3 failed"):
        srv.serve(qs)


def test_query_stream_is_seeded_and_in_range():
    a = W.serving_queries(50, rate=20.0, seed=100)
    b = W.serving_queries(50, rate=20.0, seed=100)
    assert [(q.arrival, q.m, q.steps, q.precision) for q in a] == [(q.arrival, q.m, q.steps, q.precision) for q in b]
    for q in a:
        assert q.family in ("heat", "conv") and q.m in W.SERVING_EDGES
        assert 1 <= len(q.gens) <= 8 and 1 <= len(q.C) <= 4 and 100 <= q.steps <= 2000
        assert 0.05 <= q.unsafe[0, 0] <= 1.5
        for s in [g.seg for g in q.gens] + q.C:
            assert s.lo.min() >= 0 and s.hi.max() <= q.n
    gaps = np.diff([q.arrival for q in a])
    assert np.all(gaps >= 0)


def test_cancel_waiting_and_running_queries():
    # one slot: query 0 runs (held by a gate), 1 and 2 wait.  Cancelling 1
    # while it waits keeps it from running; cancelling 0 while it runs drops
    # its verdict once it finishes; 2 runs normally; 3, cancelled before it
    # arrives, never enters the queue.
    qs = W.serving_queries(4, rate=1000.0, seed=304)
    for i, q in enumerate(qs):
        q.arrival = 0.0 if i < 3 else 0.5
    started, gate = [], threading.Event()
    lock = threading.Lock()

    def run(q, slot, keep):
        with lock:
            started.append(q.qid)
        if q.qid == qs[0].qid:
            gate.wait(5.0)
        return {"first_step": -1, "row": -1}, None, len(q.gens)
    srv = Server(None, slots=1, budget_bytes=1 << 40, runner=run, footprint=lambda q: 1)

    def client():
        while True:
            with lock:
                if started:
                    break
            time.sleep(0.001)
        srv.cancel(qs[1].qid)
        srv.cancel(qs[0].qid)
        srv.cancel(qs[3].qid)
        gate.set()
    t = threading.Thread(target=client)
    t.start()
    res = srv.serve(qs)
    t.join()
    assert started == [qs[0].qid, qs[2].qid]
    by = {r.qid: r for r in res}
    assert by[qs[0].qid].cancelled and by[qs[0].qid].verdict == {"cancelled": True}
    assert by[qs[1].qid].cancelled and by[qs[1].qid].verified_steps == 0
    assert by[qs[3].qid].cancelled
    assert not by[qs[2].qid].cancelled and by[qs[2].qid].verdict["first_step"] == -1
    s = summarize(res)
    assert s["cancelled"] == 3 and s["queries"] == 1
