"""The serving loop on the GPU: results of queries run concurrently in a mix
are bitwise identical to the same queries run alone; with batching (queries
on the same system sharing one plan) they match the queries alone to the
parity bound (FP64) or the FP32-basis bound, with the same verdicts; small
queries match the oracle; a short stream completes with every query
admitted; the box check over part of a plan's basis equals the check of a
plan of that part alone."""
import numpy as np
import pytest
import torch  # noqa: F401  (imported at collection so the first test does not pay for it)

import oracle
import workloads as W
from paper_1804_01583_amd.serve import Catalog, Server, summarize
from tests.gpu_helpers import RTOL, assert_basis_parity, require_gpu

pytestmark = pytest.mark.gpu


def _small_mix(count, max_m, seed):
    qs = [q for q in W.serving_queries(400, rate=100.0, seed=seed) if q.m <= max_m][:count]
    assert {q.family for q in qs} == {"heat", "conv"} and {q.precision for q in qs} == {"fp64", "fp32"}
    return qs


def test_alone_and_in_mix_are_identical():
    require_gpu()
    qs = _small_mix(14, 46, seed=500)
    cat = Catalog()
    cat.preload(qs)
    print(f"[gpu] serving mix of {len(qs)} queries, n <= {46 ** 3}", flush=True)
    mix = Server(cat, slots=6, batch=False).serve(qs, keep_basis=True, time_scale=0.0)   # all arrive at once
    for q, r in zip(qs, mix):
        alone = Server(cat, slots=1).serve([q], keep_basis=True, time_scale=0.0)[0]
        np.testing.assert_array_equal(r.basis, alone.basis)
        assert (r.verdict["first_step"], r.verdict["row"]) == (alone.verdict["first_step"], alone.verdict["row"])


def test_batched_queries_match_alone():
    require_gpu()
    # queries on few systems, all arriving at once: they form batches
    qs = [q for q in W.serving_queries(2000, rate=100.0, seed=504) if q.m in (22, 28)][:16]
    cat = Catalog()
    cat.preload(qs)
    print(f"[gpu] serving batches of {len(qs)} queries", flush=True)
    res = Server(cat, slots=4).serve(qs, keep_basis=True, time_scale=0.0)
    assert max(r.group for r in res) > 1
    for q, r in zip(qs, res):
        alone = Server(cat, slots=1, batch=False).serve([q], keep_basis=True, time_scale=0.0)[0]
        tol = RTOL if q.precision == "fp64" else 1e-4
        worst = assert_basis_parity(r.basis, alone.basis, rtol=tol)
        assert (r.verdict["first_step"], r.verdict["row"]) == (alone.verdict["first_step"], alone.verdict["row"])
        print(f"  query {q.qid} group {r.group} {q.precision}: {worst:.2e}", flush=True)


def test_box_check_over_part_of_a_plan():
    require_gpu()
    from paper_1804_01583_amd import kry
    p = W.small_heat3d(m=12, k=20, steps=120)
    m = 12
    gens = [W.Generator(W.box_segments((m, m, m), ((x, x + 3), (0, 4), (0, 5)), 1.0), 1.0, 0.2) for x in (0, 4, 8)]
    p.gens = gens
    p.b = None
    ds = kry.DeviceSystem(p)
    big = kry.Plan(ds)
    big.project_expm(None)
    # part: generator 1 on output rows 2 and 0, up to step 80, against a plan of that part alone
    q = W.small_heat3d(m=12, k=20, steps=80)
    q.gens, q.b = [gens[1]], None
    q.C = [p.C[2], p.C[0]]
    q.unsafe = np.array([[np.inf, np.inf], [np.inf, np.inf]])
    # both rows decay: row 0 unsafe below a threshold its lower end crosses
    # between steps 40 and 41
    lo = oracle.verify(q)["verdict"]["lo"]
    q.unsafe = np.array([[-np.inf, 0.5 * (lo[40, 0] + lo[41, 0])], [np.inf, np.inf]])
    v, z = kry.kry_check_box_subset(big.handle, [1], [2, 0], 80, q.unsafe, 1)
    small = kry.Plan(kry.DeviceSystem(q))
    small.basis()
    want = small.check(q.unsafe)
    assert (v.first_step, v.row) == (want["first_step"], want["row"]) == (41, 0)
    np.testing.assert_allclose(z, want["z"], rtol=1e-12)
    # the whole basis through the subset entry equals kry_check_box_safety
    full = big.check(p.unsafe)
    vf, zf = kry.kry_check_box_subset(big.handle, [0, 1, 2], [0, 1, 2], p.steps, p.unsafe, 3)
    assert (vf.first_step, vf.row) == (full["first_step"], full["row"])
    np.testing.assert_array_equal(zf, full["z"])
    with pytest.raises(kry.KryError):
        kry.kry_check_box_subset(big.handle, [3], [0], 10, q.unsafe[:1], 1)       # no such column
    with pytest.raises(kry.KryError):
        kry.kry_check_box_subset(big.handle, [0], [0], p.steps + 1, q.unsafe[:1], 1)
    big.close()
    small.close()


def test_small_queries_match_oracle():
    require_gpu()
    qs = [q for q in W.serving_queries(400, rate=100.0, seed=501) if q.m <= 13][:6]
    cat = Catalog()
    cat.preload(qs)
    res = Server(cat, slots=3).serve(qs, keep_basis=True, time_scale=0.0)
    for q, r in zip(qs, res):
        prob = W.query_problem(W.serving_system(q.family, q.m), q)
        ref = oracle.verify(prob)
        if q.precision == "fp64":
            tol = RTOL
        else:
            anorm = oracle.krylov.inf_norm(oracle.system_matrix(prob))
            tol = max(1e-5, 2.0 * 2.0 ** -23 * anorm * q.steps * q.dt)
        worst = assert_basis_parity(r.basis, ref["basis"], rtol=tol)
        print(f"  query {q.qid} {q.family} m={q.m} {q.precision}: {worst:.2e} (bound {tol:.0e})", flush=True)
        if q.precision == "fp64":
            assert (r.verdict["first_step"], r.verdict["row"]) == (ref["verdict"]["first_step"],
                                                                   ref["verdict"]["row"])


def test_short_stream_completes():
    require_gpu()
    qs = [q for q in W.serving_queries(200, rate=200.0, seed=502) if q.m <= 77][:40]
    cat = Catalog()
    cat.preload(qs)
    res = Server(cat, slots=8).serve(qs)
    s = summarize(res)
    print(f"  {s}", flush=True)
    assert s["queries"] == len(qs) and s["p99_ms"] > 0
