"""The serving loop on the GPU: results of queries run concurrently in a mix
are bitwise identical to the same queries run alone, small queries match the
oracle, and a short stream completes with every query admitted."""
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
    mix = Server(cat, slots=6).serve(qs, keep_basis=True, time_scale=0.0)   # all arrive at once
    for q, r in zip(qs, mix):
        alone = Server(cat, slots=1).serve([q], keep_basis=True, time_scale=0.0)[0]
        np.testing.assert_array_equal(r.basis, alone.basis)
        assert (r.verdict["first_step"], r.verdict["row"]) == (alone.verdict["first_step"], alone.verdict["row"])


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
