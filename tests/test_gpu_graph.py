"""Graph mode (kry_plan_set_graph): the projection recorded once as a HIP
graph and replayed.  Every replay, with eager work and synchronisations of
the program's own between replays, gives the eager basis bit for bit; new
input values written through the same device pointers are picked up; the
modes that read sizes back or poll the device are refused."""
import dataclasses

import numpy as np
import pytest

import workloads as W
from gpu_helpers import require_gpu

pytestmark = pytest.mark.gpu


def _eager(kry, p, ds, stream):
    plan = kry.Plan(ds, stream=stream)
    b = plan.basis()
    v = plan.check(p.unsafe)
    plan.close()
    return b, v


@pytest.mark.parametrize("name", ["heat1d", "small_heat3d", "random_arnoldi", "random_arnoldi_gram"])
def test_replays_match_eager_bitwise(name, monkeypatch):
    torch = require_gpu()
    from paper_1804_01583_amd import kry
    if name == "random_arnoldi_gram":
        # the second Gram-Schmidt pass from the Gram matrix, its guard and
        # the conditional launches recorded in the graph (the general path:
        # this size would take the persistent small-system kernel)
        monkeypatch.setenv("KRY_ARN_GS", "1")
        monkeypatch.setenv("KRY_SMALL", "0")
    if name == "heat1d":
        p = W.heat1d(steps=300)
        method = kry.KRY_AUTO
    elif name == "small_heat3d":
        p = W.small_heat3d(m=12, k=20, steps=150)
        method = kry.KRY_AUTO
    else:
        p = W.random_symmetric(n=500, k=16, steps=60, ngen=3, o=2, seed=8, affine=True, center=True)
        method = kry.KRY_ARNOLDI
    print(f"[gpu] graph {name} n={p.n}", flush=True)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        ds = kry.DeviceSystem(p)
        ref = kry.Plan(ds, stream=s, method=method)
        ref_b = ref.basis()
        ref_v = ref.check(p.unsafe)
        ref.close()
        plan = kry.Plan(ds, stream=s, method=method)
        plan.set_graph(True)
        for rep in range(4):
            b = plan.basis()
            v = plan.check(p.unsafe)
            assert np.array_equal(b, ref_b), f"replay {rep}"
            assert (v["first_step"], v["row"]) == (ref_v["first_step"], ref_v["row"])
            other = torch.ones(1 << 20, dtype=torch.float64, device="cuda") * (rep + 1)   # eager work between
            assert float(other.sum()) == float((rep + 1) << 20)
            torch.cuda.synchronize()
        plan.set_graph(False)
        b = plan.basis()
        assert np.array_equal(b, ref_b)
        plan.close()


def test_new_input_values_are_picked_up():
    torch = require_gpu()
    from paper_1804_01583_amd import kry
    p = W.small_heat3d(m=12, k=20, steps=150)
    print(f"[gpu] graph new inputs n={p.n}", flush=True)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        ds = kry.DeviceSystem(p)
        plan = kry.Plan(ds, stream=s)
        plan.set_graph(True)
        b1 = plan.basis()
        ds.b.mul_(3.0)                                   # same pointer, new forcing
        b3 = plan.basis()
        p3 = dataclasses.replace(p, b=np.asarray(p.b) * 3.0)
        ref3, _ = _eager(kry, p3, kry.DeviceSystem(p3), s)
        plan.close()
    assert np.array_equal(b3, ref3)
    assert not np.array_equal(b1, b3)


def test_refusals():
    torch = require_gpu()
    from paper_1804_01583_amd import kry
    p = W.small_heat3d(m=8, k=10, steps=20)
    print(f"[gpu] graph refusals n={p.n}", flush=True)
    ds = kry.DeviceSystem(p)
    plan = kry.Plan(ds, stream=torch.cuda.default_stream())
    with pytest.raises(kry.KryError) as ei:
        plan.set_graph(True)
    assert ei.value.status == kry.KRY_EINVAL
    plan.close()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        plan = kry.Plan(ds, stream=s)
        plan.set_error_target(1e-6)
        with pytest.raises(kry.KryError) as ei:
            plan.set_graph(True)
        assert ei.value.status == kry.KRY_ENOTSUP
        plan.close()
        plan = kry.Plan(ds, stream=s, k=80)               # dense stage
        with pytest.raises(kry.KryError) as ei:
            plan.set_graph(True)
        assert ei.value.status == kry.KRY_ENOTSUP
        plan.close()


def test_transposed_plan_replays():
    torch = require_gpu()
    from paper_1804_01583_amd import kry
    p = W.heat3d_many_inputs(m=16, k=24, steps=120)
    print(f"[gpu] graph transposed n={p.n}", flush=True)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        ds = kry.DeviceSystem(p)
        ref = kry.TransposedPlan(ds, stream=s)
        ref_b = ref.basis()
        ref.close()
        plan = kry.TransposedPlan(ds, stream=s)
        plan.set_graph(True)
        for rep in range(3):
            assert np.array_equal(plan.basis(), ref_b), f"replay {rep}"
            torch.cuda.synchronize()
        plan.close()
