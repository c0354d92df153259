"""Three-vector ("plain") projected Lanczos of Algorithm 4 at large k
(KRY_LANCZOS_PLAIN): no stored basis and no reorthogonalisation, the small
exponential in the dense stage past k = 56.  Past the loss of orthogonality
two roundings of the same process give different H_k (the copies of
converged eigenvalues land elsewhere), while the projected solution agrees
to rounding; the oracle's Lanczos is this same plain process, so parity is
checked on the basis and the verdict, with H compared only while k is small."""
import numpy as np
import pytest
import torch  # noqa: F401  (imported at collection so the first test does not pay for it)

import oracle
import workloads as W
from oracle import adaptive as AD
from paper_1804_01583_amd import kry
from tests.gpu_helpers import assert_basis_parity, assert_krylov_parity, assert_verdict_parity, gpu_verify, require_gpu
from tests.test_gpu_adaptive import _bound_tol

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True, params=["small", "general"])
def _path(request, monkeypatch):
    # every test on both FP64 Lanczos paths: the persistent small-system
    # kernel (the default up to 2048 rows) and the general launches
    if request.param == "general":
        monkeypatch.setenv("KRY_SMALL", "0")
    else:
        monkeypatch.delenv("KRY_SMALL", raising=False)


def test_plain_lanczos_large_k_matches_the_oracle():
    require_gpu()
    p = W.heat3d_paper(m=14, k=150, steps=1000)
    ref = oracle.verify(p, method="lanczos", k=150)
    got = gpu_verify(p, k=150, method=kry.KRY_LANCZOS_PLAIN)
    assert [r["k_eff"] for r in got["runs"]] == [r.k_eff for r in ref["runs"]]
    worst = assert_basis_parity(got["basis"], ref["basis"])
    assert_verdict_parity(got["verdict"], ref["verdict"], ref["basis"])
    print(f"  worst relative error {worst:.2e}", flush=True)


def test_plain_equals_lanczos_up_to_56():
    require_gpu()
    p = W.small_heat3d(m=12, k=40, steps=100)
    a = gpu_verify(p, method=kry.KRY_LANCZOS)
    b = gpu_verify(p, method=kry.KRY_LANCZOS_PLAIN)
    assert np.array_equal(a["basis"], b["basis"])
    assert_basis_parity(b["basis"], oracle.verify(p, method="lanczos")["basis"])
    # entrywise Krylov data while orthogonality holds
    q = W.small_heat3d(m=12, k=20, steps=100)
    c = gpu_verify(q, method=kry.KRY_LANCZOS_PLAIN)
    for g, r in zip(c["runs"], oracle.verify(q, method="lanczos")["runs"]):
        assert_krylov_parity(g, r)


def test_plain_lanczos_with_error_control():
    require_gpu()
    p = W.heat3d_paper(m=14, k=300, steps=1000)
    ref = AD.adaptive_verify(p, eps=1e-6, kmax=300)
    plan = kry.Plan(kry.DeviceSystem(p), k=300, method=kry.KRY_LANCZOS_PLAIN)
    plan.set_error_target(1e-6)
    basis = plan.basis()
    errs = [plan.error(r) for r in range(plan.nruns)]
    plan.close()
    r0 = ref["runs"][0]
    assert errs[0][0] == r0["k_stop"], (errs, r0["k_stop"])
    # the stop decision is well away from the target on both sides
    assert abs(r0["bound"] - 1e-6) > 1e-2 * 1e-6
    assert abs(errs[0][1] - r0["bound"]) <= _bound_tol(r0, p.steps * p.dt, ref["lam"])
    worst = assert_basis_parity(basis, ref["basis"])
    print(f"  k {errs[0][0]} bound {errs[0][1]:.3e} (oracle {r0['bound']:.3e}) worst {worst:.2e}", flush=True)


def test_plain_lanczos_is_fp64_only():
    require_gpu()
    p = W.small_heat3d(m=8, k=60, steps=10)
    with pytest.raises(kry.KryError) as ei:
        kry.Plan(kry.DeviceSystem(p), method=kry.KRY_LANCZOS_PLAIN, precision=kry.KRY_FP32_BASIS)
    assert ei.value.status == kry.KRY_ENOTSUP
