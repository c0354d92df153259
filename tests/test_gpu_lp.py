"""The per-step safety LP on the GPU (kry_check_lp_safety, Section 2.1)
against the oracle's LP (SciPy's linprog) on the oracle's basis: per-step
decisions wherever the oracle's margin is clear of rounding, the first
unsafe step, and a counter-example that satisfies every constraint."""
import json
import os

import numpy as np
import pytest

import oracle
import oracle.lp as OL
import oracle.transpose as OT
import workloads as W
from gpu_helpers import require_gpu

pytestmark = pytest.mark.gpu

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "harmonic.json")))
CLEAR = 1e-7     # decisions are compared where |margin - LP_TOL| exceeds this


def _box(p):
    return np.array([g.zc for g in p.gens]), np.array([g.radius for g in p.gens])


def _run(p, G, h, U, u, transposed=False, **kw):
    from paper_1804_01583_amd import kry
    print(f"[gpu] lp {p.name} n={p.n} ngen={len(p.gens)} o={p.o} mI={len(h)} mU={len(u)} "
          f"transposed={transposed}", flush=True)
    ds = kry.DeviceSystem(p)
    plan = kry.TransposedPlan(ds, **kw) if transposed else kry.Plan(ds, **kw)
    basis = plan.basis()
    out = plan.check_lp(G, h, U, u, flags=True)
    plan.close()
    return basis, out


def _compare(p, basis_ref, roles, G, h, U, u, got, basis_gpu, min_clear=0.9):
    zc, rad = _box(p)
    ref = OL.lp_check(basis_ref, roles, zc, rad, G, h, U, u)
    assert got["status"] == 0
    clear = np.abs(ref["margin"] - OL.LP_TOL) > CLEAR
    assert clear.mean() >= min_clear
    np.testing.assert_array_equal(got["flags"][clear], ref["feasible"][clear].astype(np.int32))
    if ref["first_step"] >= 0 and np.all(clear[:ref["first_step"] + 1]):
        assert got["first_step"] == ref["first_step"]
    if got["first_step"] >= 0:
        s = got["first_step"]
        M, f = OL.split_basis(basis_gpu[s], roles)
        z = got["z"]
        assert np.all(z >= zc - rad - 1e-12) and np.all(z <= zc + rad + 1e-12)
        # no row, scaled to a largest coefficient of 1, is violated by more
        # than the LP tolerance
        A = np.vstack([np.reshape(G, (len(h), len(zc))), U @ M])
        b = np.concatenate([h, u - U @ f])
        sc = np.abs(A).max(axis=1) if len(zc) else np.zeros(len(b))
        sc[sc == 0.0] = 1.0
        assert np.all((A @ z - b) / sc <= OL.LP_TOL + 1e-9)
        y = M @ z + f
        np.testing.assert_allclose(got["y"], y, rtol=1e-12, atol=1e-12)
    return ref


def test_worked_example():
    require_gpu()
    p = W.harmonic_oscillator()
    U, u = np.array([[1.0], [-1.0]]), np.array([4.0, -4.0])
    basis, got = _run(p, np.zeros((0, 1)), np.zeros(0), U, u)
    ref = oracle.verify(p)
    # the unsafe set is the line x = 4: the deciding step touches it with no
    # interior (margin 0), so only the other steps are compared by margin
    _compare(p, ref["basis"], ref["roles"], np.zeros((0, 1)), np.zeros(0), U, u, got, basis, min_clear=0.8)
    assert got["first_step"] == GOLD["verdicts"]["unsafe_first_step"]
    np.testing.assert_allclose(got["z"][0], GOLD["counter_example"]["x0"][1], atol=5e-3)
    np.testing.assert_allclose(got["y"], [4.0], atol=1e-9)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_polytope_and_halfspaces(seed):
    require_gpu()
    p = W.random_symmetric(n=300, k=12, steps=200, dt=0.05, ngen=3, o=2, seed=seed, affine=True, center=True)
    ref = oracle.verify(p)
    rng = np.random.default_rng(100 + seed)
    zc, rad = _box(p)
    G = rng.normal(0, 1, (2, 3)); h = G @ zc + rng.uniform(0.0, 0.3, 2)
    # unsafe: both outputs beyond a level the trajectory crosses
    lvl = np.quantile(ref["basis"][:, :, :].sum(axis=2), 0.3, axis=0)
    U = np.array([[-1.0, 0.0], [0.0, -1.0], [1.0, 1.0]]); u = np.array([-lvl[0], -lvl[1], 50.0])
    basis, got = _run(p, G, h, U, u)
    _compare(p, ref["basis"], ref["roles"], G, h, U, u, got, basis)


def test_sixteen_generators():
    require_gpu()
    p = W.random_symmetric(n=400, k=14, steps=150, dt=0.05, ngen=16, o=3, seed=9, affine=True, center=False)
    ref = oracle.verify(p)
    rng = np.random.default_rng(9)
    zc, rad = _box(p)
    G = rng.normal(0, 1, (20, 16)); h = G @ zc + rng.uniform(0.05, 0.5, 20)
    mid = ref["basis"].sum(axis=2)
    U = rng.normal(0, 1, (6, 3)); u = np.quantile(mid @ U.T, 0.6, axis=0)
    basis, got = _run(p, G, h, U, u)
    _compare(p, ref["basis"], ref["roles"], G, h, U, u, got, basis)


def test_transposed_plan_many_inputs():
    require_gpu()
    p = W.heat3d_many_inputs(m=20, k=30, steps=300)
    ref = OT.verify_transposed(p)
    d = len(p.gens)
    G = np.ones((1, d)); h = np.array([d * 1.0 + 0.05])          # the generators' sum is capped
    U = np.array([[1.0]]); u = np.array([0.4])                   # the warm cube's mean at or below 0.4
    basis, got = _run(p, G, h, U, u, transposed=True)
    r = _compare(p, ref["basis"], ref["roles"], G, h, U, u, got, basis)
    assert r["first_step"] > 0


def test_whole_output_space_unsafe_and_empty_initial_set():
    require_gpu()
    p = W.random_symmetric(n=100, k=10, steps=20, dt=0.05, ngen=2, o=1, seed=4)
    zc, rad = _box(p)
    # no unsafe constraint: every state is unsafe, so step 0 is
    _, got = _run(p, np.zeros((0, 2)), np.zeros(0), np.zeros((0, 1)), np.zeros(0))
    assert got["first_step"] == 0 and np.all(got["flags"] == 1)
    # an initial polytope outside the box: never unsafe
    G = np.array([[1.0, 0.0]]); h = np.array([zc[0] - rad[0] - 0.1])
    _, got = _run(p, G, h, np.zeros((0, 1)), np.zeros(0))
    assert got["first_step"] == -1 and np.all(got["flags"] == 0)


def test_point_initial_set_and_no_generators():
    # every radius 0: the initial set is one point; and a plan without
    # generators (center and forcing only) decides U f_s <= u alone
    require_gpu()
    import dataclasses
    p = W.random_symmetric(n=300, k=12, steps=120, dt=0.05, ngen=3, o=2, seed=6, affine=True, center=True)
    p = dataclasses.replace(p, gens=[dataclasses.replace(g, radius=0.0) for g in p.gens])
    ref = oracle.verify(p)
    lvl = np.quantile(ref["basis"].sum(axis=2), 0.5, axis=0)
    U = np.array([[-1.0, 0.0], [0.0, -1.0]]); u = -lvl
    basis, got = _run(p, np.zeros((0, 3)), np.zeros(0), U, u)
    r = _compare(p, ref["basis"], ref["roles"], np.zeros((0, 3)), np.zeros(0), U, u, got, basis)
    np.testing.assert_array_equal(got["z"], [g.zc for g in p.gens] if got["first_step"] >= 0 else got["z"])
    q = dataclasses.replace(p, gens=[])
    refq = oracle.verify(q)
    basis, got = _run(q, np.zeros((0, 0)), np.zeros(0), U, u)
    _compare(q, refq["basis"], refq["roles"], np.zeros((0, 0)), np.zeros(0), U, u, got, basis)


def test_block_arnoldi_plan():
    # sixteen generators advanced as one block Krylov space, then the LP
    require_gpu()
    from paper_1804_01583_amd import kry
    import oracle.block as OB
    p = W.conv_diff3d(nx=12, ny=12, nz=14, ngen=16, gen_len=20, o=3, k=6, dt=1e-3, steps=60)
    ref = OB.block_verify(p, p=16)
    rng = np.random.default_rng(3)
    zc, rad = _box(p)
    G = rng.normal(0, 1, (4, 16)); h = G @ zc + rng.uniform(0.05, 0.3, 4)
    mid = ref["basis"].sum(axis=2)
    U = rng.normal(0, 1, (3, 3)); u = np.quantile(mid @ U.T, 0.5, axis=0)
    basis, got = _run(p, G, h, U, u, method=kry.KRY_BLOCK_ARNOLDI, block_p=16)
    _compare(p, ref["basis"], ref["roles"], G, h, U, u, got, basis)
