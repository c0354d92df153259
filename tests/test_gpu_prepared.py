"""Prepared matrices (kry_matrix_create): a CSR system's sliced-ELL copy and
norm built once and shared by plans.  A plan that uses one computes exactly
what a plan that builds its own computes (same copy, same norm, same
kernels), so results are compared bit for bit."""
import numpy as np
import pytest
import torch  # noqa: F401  (imported at collection so the first test does not pay for it)

import workloads as W
from paper_1804_01583_amd import kry
from tests.gpu_helpers import require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _general_path(monkeypatch):
    # these kernels belong to the general path: small systems would take the
    # persistent small-system kernel instead
    monkeypatch.setenv("KRY_SMALL", "0")


def _same_verdict(a, b):
    return a.keys() == b.keys() and all(np.array_equal(np.asarray(a[k]), np.asarray(b[k])) for k in a)


def _run(dsys, **kw):
    plan = kry.Plan(dsys, **kw)
    basis = plan.basis()
    verdict = plan.check(dsys.problem.unsafe)
    runs = [plan.krylov(r) for r in range(plan.nruns)] if kw.get("method") != kry.KRY_BLOCK_ARNOLDI else None
    plan.close()
    return basis, verdict, runs


@pytest.mark.parametrize("precision", [kry.KRY_FP64, kry.KRY_FP32_BASIS])
def test_prepared_matrix_gives_identical_results(precision):
    require_gpu()
    p = W.small_heat3d(m=12, k=30, steps=80)
    print(f"[gpu] prepared {p.name} n={p.n} precision={precision}", flush=True)
    own = kry.DeviceSystem(p)
    b0, v0, r0 = _run(own, precision=precision)
    shared = kry.DeviceSystem(p)
    shared.prepare(precision)
    b1, v1, r1 = _run(shared, precision=precision)
    b2, v2, r2 = _run(shared, precision=precision)          # a second plan on the same copy
    assert np.array_equal(b0, b1) and np.array_equal(b1, b2)
    assert _same_verdict(v0, v1) and _same_verdict(v1, v2)
    for a, b in zip(r0, r1):
        assert a["k_eff"] == b["k_eff"] and np.array_equal(a["H"], b["H"]) and np.array_equal(a["P"], b["P"])
    shared.close()


def test_prepared_matrix_with_arnoldi_block_and_error_control():
    require_gpu()
    p = W.conv_diff3d(10, 10, 12, ngen=4, gen_len=30, o=3, k=12, steps=40, dt=1e-3, seed=6)
    own = kry.DeviceSystem(p)
    shared = kry.DeviceSystem(p)
    shared.prepare(kry.KRY_FP64)
    for method in (kry.KRY_ARNOLDI, kry.KRY_BLOCK_ARNOLDI):
        b0, v0, _ = _run(own, method=method)
        b1, v1, _ = _run(shared, method=method)
        assert np.array_equal(b0, b1) and _same_verdict(v0, v1)
    q = W.small_heat3d(m=10, k=40, steps=60)
    own, shared = kry.DeviceSystem(q), kry.DeviceSystem(q)
    shared.prepare(kry.KRY_FP64)
    out = []
    for ds in (own, shared):
        plan = kry.Plan(ds)
        plan.set_error_target(1e-7)
        out.append((plan.basis(), [plan.error(r) for r in range(plan.nruns)]))
        plan.close()
    assert np.array_equal(out[0][0], out[1][0]) and out[0][1] == out[1][1]
    shared.close()


def test_prepared_matrix_rejects_other_precision_and_system():
    require_gpu()
    p = W.small_heat3d(m=8, k=10, steps=10)
    ds = kry.DeviceSystem(p)
    ds.prepare(kry.KRY_FP64)
    # a plan of the other precision with this matrix named explicitly
    s = kry.KrySystem.from_buffer_copy(ds.sys)
    s.prepared = ds.prepared[kry.KRY_FP64]
    keep = []
    gens = [kry.KryGen(kry._segs(g.seg, keep), g.zc, g.radius) for g in p.gens]
    C = [kry._segs(c, keep) for c in p.C]
    with pytest.raises(kry.KryError) as ei:
        kry.kry_plan_create(s, gens, None, C, 10, p.dt, p.steps, kry.KRY_FP32_BASIS, kry.KRY_AUTO, 0, None, 0, None)
    assert ei.value.status == kry.KRY_EINVAL
    # the matrix of another system
    other = kry.DeviceSystem(W.small_heat3d(m=8, k=10, steps=10))
    s2 = kry.KrySystem.from_buffer_copy(other.sys)
    s2.prepared = ds.prepared[kry.KRY_FP64]
    with pytest.raises(kry.KryError) as ei:
        kry.kry_plan_create(s2, gens, None, C, 10, p.dt, p.steps, kry.KRY_FP64, kry.KRY_AUTO, 0, None, 0, None)
    assert ei.value.status == kry.KRY_EINVAL
    ds.close()


def test_footprint_leaves_the_prepared_copy_out():
    require_gpu()
    p = W.small_heat3d(m=40, k=20, steps=50)
    ds = kry.DeviceSystem(p)
    nseg = sum(g.seg.nseg for g in p.gens) + sum(c.nseg for c in p.C)
    own = kry.kry_plan_workspace(ds.sys, 2, len(p.C), p.k, p.steps, nseg)
    h = ds.prepare(kry.KRY_FP64)
    shared = kry.kry_plan_workspace(ds.system_for(kry.KRY_FP64), 2, len(p.C), p.k, p.steps, nseg)
    mbytes = kry.kry_matrix_bytes(h)
    # FP64 values and 16-bit column offsets (every column is within 1600 of
    # its row here); a plan that builds its own copy reserves 32-bit columns
    assert mbytes >= 10 * p.nnz
    assert own - shared >= 12 * p.nnz
    ds.close()
