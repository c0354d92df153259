"""Parity at the sizes and in the launch configuration the benchmark times:
the 100^3 heat system (n = 10^6, CSR, forcing, Lanczos k = 40, 2000 steps,
FP64) with its matrix prepared once, the eight-column 100^3 heat system by
the transposed route, and the per-step LP on it.  The oracle finishes each
in a few seconds, so every output is compared."""
import numpy as np
import pytest

import oracle
import oracle.lp as OL
import oracle.transpose as OT
import workloads as W
from gpu_helpers import assert_basis_parity, assert_verdict_parity, require_gpu

pytestmark = pytest.mark.gpu


def test_heat3d_100_full_size_prepared():
    require_gpu()
    from paper_1804_01583_amd import kry
    p = W.heat3d_csr()
    print(f"[gpu] bench size {p.name} n={p.n} k={p.k} steps={p.steps}", flush=True)
    ds = kry.DeviceSystem(p)
    ds.prepare()
    plan = kry.Plan(ds)
    basis = plan.basis()
    v = plan.check(p.unsafe)
    plan.close()
    ds.close()
    ref = oracle.verify(p)
    assert_basis_parity(basis, ref["basis"])
    assert_verdict_parity(v, ref["verdict"], ref["basis"])


def test_eight_columns_transposed_full_size_with_lp():
    require_gpu()
    import bench
    from paper_1804_01583_amd import kry
    p = W.heat3d_many_inputs()
    print(f"[gpu] bench size {p.name} n={p.n} k={p.k} steps={p.steps}", flush=True)
    ds = kry.DeviceSystem(p)
    ds.prepare()
    plan = kry.TransposedPlan(ds)
    basis = plan.basis()
    v = plan.check(p.unsafe)
    G, h, U, u = bench.lp_sets(p)
    lp = plan.check_lp(G, h, U, u, flags=True)
    plan.close()
    ds.close()
    ref = OT.verify_transposed(p)
    assert_basis_parity(basis, ref["basis"])
    assert_verdict_parity(v, ref["verdict"], ref["basis"])
    zc = np.array([g.zc for g in p.gens]); rad = np.array([g.radius for g in p.gens])
    rl = OL.lp_check(ref["basis"], ref["roles"], zc, rad, G, h, U, u)
    clear = np.abs(rl["margin"] - OL.LP_TOL) > 1e-7
    assert clear.mean() > 0.99
    np.testing.assert_array_equal(lp["flags"][clear], rl["feasible"][clear].astype(np.int32))
    assert lp["first_step"] == rl["first_step"]
