"""Pins of the per-step safety LP (Section 2.1) in oracle/lp.py: the
worked example's unique counter-example, agreement with the exact box
check when the sets reduce to a box and an interval, brute-force vertex
enumeration on small polytopes, and the margin's sign."""
import itertools
import json
import os

import numpy as np
import pytest

import oracle
import oracle.lp as OL
import workloads as W

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "harmonic.json")))


def test_worked_example_counter_example():
    # unsafe x = 4 as two halfspaces x <= 4, -x <= -4; initial y0 in [0, 1]
    p = W.harmonic_oscillator()
    res = oracle.verify(p)
    g = p.gens[0]
    out = OL.lp_check(res["basis"], res["roles"], [g.zc], [g.radius], np.zeros((0, 1)), np.zeros(0),
                      np.array([[1.0], [-1.0]]), np.array([4.0, -4.0]))
    assert out["first_step"] == GOLD["verdicts"]["unsafe_first_step"]
    assert not out["feasible"][:3].any()
    # x(t) = -5 cos t + y0 sin t = 4 has one solution y0 at t = 3 pi / 4
    np.testing.assert_allclose(out["z"][0], GOLD["counter_example"]["x0"][1], atol=5e-3)
    np.testing.assert_allclose(out["y"], [4.0], atol=1e-7)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_box_and_interval_reduce_to_the_box_check(seed):
    # one output row, interval unsafe set [lo, hi] = {y <= hi, -y <= -lo},
    # initial set the generator box: the LP decides exactly as the range check
    p = W.random_symmetric(n=80, k=12, steps=40, dt=0.05, ngen=3, o=1, seed=seed, affine=True, center=True)
    res = oracle.verify(p)
    rng = np.random.default_rng(seed)
    mid = res["basis"][:, 0, :].sum(axis=1)
    lo = float(np.quantile(mid, 0.5)) + 0.01 * rng.uniform()
    hi = lo + 0.05
    zc = np.array([g.zc for g in p.gens]); rad = np.array([g.radius for g in p.gens])
    box = oracle.box_check(res["basis"], res["roles"], zc, rad, np.array([[lo, hi]]))
    out = OL.lp_check(res["basis"], res["roles"], zc, rad, np.zeros((0, 3)), np.zeros(0),
                      np.array([[1.0], [-1.0]]), np.array([hi, -lo]))
    # compare where the range is not within the LP tolerance of the interval
    # ends (the LP errs towards unsafe by at most LP_TOL on scaled rows)
    clear = (np.abs(out["margin"] - OL.LP_TOL) > 1e-7)
    assert clear.sum() > 30
    np.testing.assert_array_equal(out["feasible"][clear], box["unsafe_mask"][clear, 0])
    assert out["first_step"] == box["first_step"]
    np.testing.assert_array_equal(out["feasible"][out["margin"] < -1e-7], True)


def _brute_force_feasible(A, b):
    """Non-empty {x : A x <= b} for a bounded set: some vertex (a solution of
    d active rows) satisfies every row."""
    m, d = A.shape
    for rows in itertools.combinations(range(m), d):
        Asub = A[list(rows)]
        if abs(np.linalg.det(Asub)) < 1e-12:
            continue
        x = np.linalg.solve(Asub, b[list(rows)])
        if np.all(A @ x <= b + 1e-9):
            return True
    return False


@pytest.mark.parametrize("d", [1, 2, 3])
def test_polytopes_against_vertex_enumeration(d):
    rng = np.random.default_rng(10 + d)
    checked = 0
    for trial in range(60):
        o = int(rng.integers(1, 3))
        M = rng.normal(0, 1, (o, d)); f = rng.normal(0, 0.5, o)
        zc = rng.normal(0, 1, d); rad = rng.uniform(0.2, 1.0, d)
        mI, mU = int(rng.integers(0, 3)), int(rng.integers(1, 4))
        G = rng.normal(0, 1, (mI, d)); h = G @ zc + rng.uniform(-0.3, 0.8, mI)
        U = rng.normal(0, 1, (mU, o)); u = rng.normal(0, 1, mU)
        margin = OL.lp_margin(M, f, zc - rad, zc + rad, G, h, U, u)
        if abs(margin) < 1e-6:
            continue
        ok, z = OL.lp_feasible(M, f, zc - rad, zc + rad, G, h, U, u)
        A = np.vstack([np.eye(d), -np.eye(d), G, U @ M])
        b = np.concatenate([zc + rad, -(zc - rad), h, u - U @ f])
        assert ok == _brute_force_feasible(A, b)
        assert ok == (margin < 0)
        if ok:
            assert np.all(A @ z <= b + 1e-9)
        checked += 1
    assert checked >= 40


def test_empty_initial_polytope_is_never_unsafe():
    # G z <= h excludes the whole box: no step can be unsafe
    p = W.random_symmetric(n=60, k=8, steps=10, dt=0.05, ngen=2, o=1, seed=4)
    res = oracle.verify(p)
    zc = np.array([g.zc for g in p.gens]); rad = np.array([g.radius for g in p.gens])
    G = np.array([[1.0, 0.0]]); h = np.array([zc[0] - rad[0] - 0.1])
    out = OL.lp_check(res["basis"], res["roles"], zc, rad, G, h, np.array([[1.0]]), np.array([1e9]))
    assert out["first_step"] == -1 and not out["feasible"].any()
    # without it, the same unsafe halfspace (y <= 1e9) holds at step 0
    out = OL.lp_check(res["basis"], res["roles"], zc, rad, np.zeros((0, 2)), np.zeros(0), np.array([[1.0]]),
                      np.array([1e9]))
    assert out["first_step"] == 0
