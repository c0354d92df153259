"""Failure handling on the GPU: a non-finite value in the matrix, the
forcing or the center reaches the basis and the verdict reports
KRY_ENUMERIC (the boundary's contract for non-finite inputs) while runs
that never touch it keep their finite result; a plan too large for device
memory gives KRY_ENOMEM from the library's own allocation; a kry_plan
created through the boundary's short form behaves like kry_plan_create."""
import math

import numpy as np
import pytest
import torch  # noqa: F401  (imported at collection so the first test does not pay for it)

import oracle
import workloads as W
from paper_1804_01583_amd import kry
from tests.gpu_helpers import assert_basis_parity, gpu_verify, require_gpu

pytestmark = pytest.mark.gpu


def _poisoned(p, where, value):
    p = W.small_heat3d(m=10, k=20, steps=60) if p is None else p
    if where == "A":
        p.vals = p.vals.copy()
        p.vals[len(p.vals) // 3] = value
    elif where == "b":
        p.b = p.forcing().copy()
        p.b_seg = None
        nz = np.flatnonzero(p.b)
        p.b[nz[len(nz) // 2]] = value
    elif where == "center":
        c = np.zeros(p.n)
        c[:50] = 0.5
        c[7] = value
        p.center = c
    return p


@pytest.mark.parametrize("where,value", [("A", math.nan), ("A", math.inf), ("b", math.nan), ("center", math.nan),
                                         ("center", -math.inf)])
def test_non_finite_input_gives_enumeric_verdict(where, value):
    require_gpu()
    p = _poisoned(None, where, value)
    print(f"[gpu] fault {where}={value} n={p.n}", flush=True)
    got = gpu_verify(p)
    assert got["verdict"]["status"] == kry.KRY_ENUMERIC
    roles = got["roles"]
    if where != "A":
        # the generator run never reads the poisoned vector
        clean = _poisoned(None, where, 0.0)
        ref = oracle.verify(clean)
        g = [i for i, r in enumerate(roles) if r == "gen"]
        assert np.isfinite(got["basis"][:, :, g]).all()
        assert_basis_parity(got["basis"][:, :, g], ref["basis"][:, :, g])
        bad = roles.index("affine" if where == "b" else "center")
        assert not np.isfinite(got["basis"][:, :, bad]).all()


def test_non_finite_matrix_in_the_dense_stage():
    # k > 56: the run's exponential goes through the dense stage, which
    # marks the run's columns non-finite instead of failing the call
    require_gpu()
    p = _poisoned(W.small_heat3d(m=10, k=80, steps=40), "A", math.nan)
    print(f"[gpu] fault dense stage n={p.n} k={p.k}", flush=True)
    got = gpu_verify(p, method=kry.KRY_LANCZOS_PLAIN)
    assert got["verdict"]["status"] == kry.KRY_ENUMERIC


def test_plan_beyond_device_memory_gives_enomem():
    # a 3000^3 matrix-free system: three FP64 vectors per run alone exceed
    # the device's memory, so the library's own hipMalloc fails cleanly
    require_gpu()
    p = W.heat3d_stencil(m=3000, k=20, steps=10)
    need = kry.kry_footprint(kry.DeviceSystem(p).sys, len(p.gens), len(p.C), p.k)
    assert need > 300 * 2**30
    print(f"[gpu] enomem n={p.n} footprint {need / 2**30:.0f} GiB", flush=True)
    with pytest.raises(kry.KryError) as ei:
        kry.Plan(kry.DeviceSystem(p), workspace="library")
    assert ei.value.status == kry.KRY_ENOMEM
    # the library keeps working afterwards
    small = W.small_heat3d(m=8, k=12, steps=20)
    assert_basis_parity(gpu_verify(small)["basis"], oracle.verify(small)["basis"])


def test_kry_plan_short_form_matches_plan_create():
    require_gpu()
    p = W.small_heat3d(m=10, k=20, steps=60)
    ds = kry.DeviceSystem(p)
    keep = []
    gens = [kry.KryGen(kry._segs(g.seg, keep), g.zc, g.radius) for g in p.gens]
    rows = [kry._segs(c, keep) for c in p.C]
    h = kry.kry_plan(ds.sys, gens, None, rows, p.k, p.dt, p.steps)
    try:
        out = torch.zeros((p.steps + 1, len(p.C), 2), dtype=torch.float64)
        kry.kry_project_expm(h, out.data_ptr())
        v, _ = kry.kry_check_box_safety(h, p.unsafe, len(p.gens))
    finally:
        kry.kry_plan_destroy(h)
    ref = gpu_verify(p)
    assert np.array_equal(out.numpy(), ref["basis"])
    assert v.first_step == ref["verdict"]["first_step"]


def test_zero_generator_in_the_dense_stage():
    # k > 56 sends every run through the dense stage; a zero generator has
    # no Krylov space there either and its column is exactly zero
    require_gpu()
    p = W.heat1d(steps=50)
    p.k = 80
    p.gens = [W.Generator(W.segments_from_ranges([(0, 5)], 0.0), 0.0, 1.0),
              W.Generator(W.segments_from_ranges([(0, 10)], 1.0), 0.0, 0.1)]
    p.C = [W.segments_from_ranges([(0, 30)], 1.0 / 30.0)]
    p.unsafe = np.array([[0.9, math.inf]])
    print(f"[gpu] zero generator dense stage n={p.n} k={p.k}", flush=True)
    got = gpu_verify(p)
    ref = oracle.verify(p)
    assert [r["k_eff"] for r in got["runs"]][0] == 0
    assert np.all(got["basis"][:, :, 0] == 0.0)
    assert_basis_parity(got["basis"], ref["basis"])
    assert got["verdict"]["status"] == kry.KRY_OK
