"""kry_verify_noalloc: plan, projection and box check in one call on the
library's fixed scratch array (for callers that cannot allocate device
memory).  Its basis and verdict must equal those of kry_plan_create with a
caller workspace (the same kernels on the same sizes: bit for bit), on two
calls in a row, the second one smaller, so the second call runs on the
first one's leftovers."""
import math

import numpy as np
import pytest
import torch

import workloads as W
from paper_1804_01583_amd import kry
from tests.gpu_helpers import require_gpu

pytestmark = pytest.mark.gpu


def _noalloc(p, dsys):
    keep = []
    gens = [kry.KryGen(kry._segs(g.seg, keep), float(g.zc), float(g.radius)) for g in p.gens]
    rows = [kry._segs(c, keep) for c in p.C]
    nruns = len(p.gens) + (dsys.center is not None) + (dsys.b is not None or p.b_seg is not None)
    out = torch.full((p.steps + 1, len(p.C), nruns), math.nan, dtype=torch.float64, device=dsys.device)
    stream = torch.cuda.current_stream(dsys.device)
    v, z = kry.kry_verify_noalloc(dsys.system_for(kry.KRY_FP64), gens, kry._ptr(dsys.center), rows, p.k, p.dt,
                                  p.steps, np.asarray(p.unsafe, np.float64), out.data_ptr(),
                                  stream_ptr=stream.cuda_stream)
    torch.cuda.synchronize()
    return out.cpu().numpy(), v, z


def _with_plan(dsys):
    plan = kry.Plan(dsys)
    basis = plan.basis()
    verdict = plan.check(dsys.problem.unsafe)
    plan.close()
    return basis, verdict


def _case(p):
    require_gpu()
    dsys = kry.DeviceSystem(p)
    print(f"[gpu] noalloc {p.name} n={p.n} k={p.k} steps={p.steps}", flush=True)
    got, v, z = _noalloc(p, dsys)
    ref, verdict = _with_plan(dsys)
    assert np.array_equal(got, ref)
    assert v.first_step == verdict["first_step"] and v.row == verdict["row"]
    assert v.status == verdict["status"]
    np.testing.assert_array_equal(z, verdict["z"])
    return v


def test_noalloc_matches_plan_twice_second_smaller():
    big = W.small_heat3d(m=14, k=24, steps=120)
    c = np.zeros(big.n)
    c[:40] = 0.25
    big.center = c
    # row 1 (the forcing cube's mean) starts near 0 and reaches 0.01 after a
    # few steps: the first violation and its counter-example are compared too
    big.unsafe = np.array([[math.inf, math.inf]] * big.o)
    big.unsafe[1, 0] = 0.01
    first = _case(big)
    assert first.first_step >= 0
    small = W.small_heat3d(m=8, k=12, steps=40)
    _case(small)


def test_noalloc_stencil_and_dense_stage():
    require_gpu()
    p = W.small_heat3d(m=10, k=20, steps=60)
    ps = W.Problem("stencil", p.n, "stencil7", True, p.gens, p.C, p.unsafe, k=70, dt=p.dt, steps=p.steps,
                   b=p.b, grid=(10, 10, 10), coef=p.meta["coef"])
    _case(ps)                      # k > 56: the dense small stage
    _case(W.small_heat3d(m=6, k=10, steps=30))


def test_noalloc_rejects_sizes_beyond_the_scratch_array():
    require_gpu()
    p = W.heat3d_stencil(m=300, k=20, steps=10)
    dsys = kry.DeviceSystem(p)
    need = kry.kry_plan_workspace(dsys.sys, 2, len(p.C), p.k, p.steps,
                                  sum(g.seg.nseg for g in p.gens) + sum(c.nseg for c in p.C) + 1, kry.KRY_FP64,
                                  kry.KRY_AUTO, 0)
    assert need > kry.KRY_NOALLOC_SCRATCH_BYTES
    with pytest.raises(kry.KryError) as ei:
        _noalloc(p, dsys)
    assert ei.value.status == kry.KRY_ENOMEM
    # the entry point keeps working afterwards
    _case(W.small_heat3d(m=8, k=12, steps=40))
