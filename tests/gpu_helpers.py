"""Shared helpers of the GPU tests: run a problem through the C ABI and
compare with the oracle."""
import contextlib
import os

import numpy as np
import pytest

# FP64 parity bound: per (output row, run), max over steps of |gpu - oracle|
# must stay within this fraction of max over steps of |oracle|.
RTOL = 1e-10


def require_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    from paper_1804_01583_amd import kry   # noqa: F401  (fails loudly if the library is missing)
    return torch


def gpu_verify(problem, **kw):
    """Plan + project + check on the GPU; returns dict like oracle.verify."""
    from paper_1804_01583_amd import kry
    print(f"[gpu] {problem.name} n={problem.n} k={kw.get('k', problem.k)} steps={kw.get('steps', problem.steps)} "
          f"kw={ {k: v for k, v in kw.items() if k != 'dsys'} }", flush=True)
    dsys = kw.pop("dsys", None) or kry.DeviceSystem(problem)
    plan = kry.Plan(dsys, **kw)
    basis = plan.basis()
    verdict = plan.check(problem.unsafe)
    runs = [plan.krylov(r) for r in range(plan.nruns)]
    roles = list(plan.roles)
    plan.close()
    return {"basis": basis, "verdict": verdict, "runs": runs, "roles": roles}


def assert_basis_parity(got, ref, rtol=RTOL):
    assert got.shape == ref.shape, (got.shape, ref.shape)
    S1, o, nr = ref.shape
    worst = 0.0
    for q in range(o):
        for r in range(nr):
            a, b = got[:, q, r], ref[:, q, r]
            scale = np.abs(b).max()
            if scale == 0.0:
                assert np.all(a == 0.0), f"row {q} run {r}: oracle is structurally zero, gpu max {np.abs(a).max()}"
                continue
            err = np.abs(a - b).max() / scale
            worst = max(worst, err)
            assert err <= rtol, f"row {q} run {r}: relative error {err:.3e} > {rtol:.1e}"
    return worst


def assert_krylov_parity(gpu_run, ref_run, rtol=RTOL):
    assert gpu_run["k_eff"] == ref_run.k_eff
    if ref_run.k_eff == 0:
        return
    assert abs(gpu_run["beta0"] - ref_run.beta0) <= 1e-13 * abs(ref_run.beta0)
    Hs = np.abs(ref_run.H).max()
    np.testing.assert_allclose(gpu_run["H"], ref_run.H, rtol=0, atol=rtol * Hs)
    Ps = np.abs(ref_run.P).max()
    if Ps == 0:
        assert np.all(gpu_run["P"] == 0)
    else:
        np.testing.assert_allclose(gpu_run["P"], ref_run.P, rtol=0, atol=rtol * Ps)


def assert_verdict_parity(gv, ov, basis, tol=1e-9):
    """Same first violation; the counter-example lands in the unsafe set.
    A decision is only compared when its margin exceeds tol * scale."""
    assert gv["status"] == 0
    if ov["first_step"] == -1:
        assert gv["first_step"] == -1
        return
    assert (gv["first_step"], gv["row"]) == (ov["first_step"], ov["row"])
    np.testing.assert_allclose(gv["z"], ov["z"], rtol=1e-8, atol=1e-10)
    assert abs(gv["y"] - ov["y"]) <= tol * max(1.0, abs(ov["y"]))


@contextlib.contextmanager
def env(**kv):
    """Environment variables set for the duration of a with-block (the
    library reads its switches when a plan projects)."""
    old = {k: os.environ.get(k) for k in kv}
    os.environ.update(kv)
    try:
        yield
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
