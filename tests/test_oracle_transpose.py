"""Pins of the transposed route (Section 4.1) in oracle/transpose.py: the
paper's worked example, brute force against a dense exponential of the
augmented system, a diagonal closed form, the Krylov error at k < n, and
agreement with the forward route where both are exact."""
import json
import math
import os

import numpy as np
import scipy.linalg
import scipy.sparse as sp

import oracle
import oracle.transpose as OT
import workloads as W

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "harmonic.json")))


def _problem_from_dense(A, gens, C, k, dt, steps, b=None, center=None, symmetric=False):
    A = np.asarray(A, np.float64)
    n = A.shape[0]
    nzr, nzc = np.nonzero(A)
    rowptr = np.zeros(n + 1, np.int64)
    np.add.at(rowptr, nzr + 1, 1)
    rowptr = np.cumsum(rowptr)
    unsafe = np.stack([np.full(len(C), 1e30), np.full(len(C), math.inf)], axis=1)
    return W.Problem("dense", n, "csr", symmetric, gens, C, unsafe, k=k, dt=dt, steps=steps, b=b, center=center,
                     rowptr=rowptr, colidx=nzc.astype(np.int32), vals=A[nzr, nzc])


def _dense_basis(p, s_list):
    """C e^{A~ t} E by a dense exponential of the augmented matrix (SciPy)."""
    n = p.n
    A = oracle.system_matrix(p).toarray()
    cols = [g.seg.dense(n) for g in p.gens]
    if p.center is not None:
        cols.append(np.asarray(p.center, float))
    Cm = np.stack([c.dense(n) for c in p.C])
    if p.has_forcing:
        Aa = np.zeros((n + 1, n + 1)); Aa[:n, :n] = A; Aa[:n, n] = p.forcing()
        E = np.zeros((n + 1, len(cols) + 1))
        for j, c in enumerate(cols):
            E[:n, j] = c
        E[n, -1] = 1.0
        Ca = np.hstack([Cm, np.zeros((Cm.shape[0], 1))])
    else:
        Aa, E, Ca = A, np.stack(cols, axis=1), Cm
    return np.stack([Ca @ scipy.linalg.expm(Aa * (s * p.dt)) @ E for s in s_list])


def test_worked_example_by_transposed_simulation():
    # Section 4.1: one simulation of A^T from the output direction gives the
    # whole basis row (0.707, 3.54) at t = 3 pi / 4
    p = W.harmonic_oscillator()
    res = OT.verify_transposed(p)
    assert res["roles"] == ["gen", "center", "affine"]
    assert len(res["runs"]) == 1
    M = res["basis"][3, 0]
    paper = GOLD["projected_basis_CeAtE_at_3pi_over_4"]["row"]
    np.testing.assert_allclose([M[0], M[1] + M[2]], paper, atol=5e-3)
    v = res["verdict"]
    assert v["first_step"] == GOLD["verdicts"]["unsafe_first_step"]
    np.testing.assert_allclose(v["z"][0], GOLD["counter_example"]["x0"][1], atol=5e-3)


def test_nonsymmetric_affine_matches_dense_exponential():
    # k = n: the Krylov space of A^T is the whole space and the route is exact
    rng = np.random.default_rng(3)
    n = 7
    A = rng.normal(0, 1, (n, n)) * (rng.uniform(size=(n, n)) < 0.6) - 1.5 * np.eye(n)
    gens = [W.Generator(W.segments_from_ranges([(0, 2)], 0.7), 0.2, 0.1),
            W.Generator(W.segments_from_ranges([(3, 4), (5, 7)], -1.3), -0.4, 0.3),
            W.Generator(W.segments_from_ranges([(2, 3)], 2.0), 1.0, 0.5)]
    C = [W.segments_from_ranges([(1, 5)], 0.25), W.segments_from_ranges([(0, 1), (6, 7)], 1.0)]
    b = rng.normal(0, 1, n)
    center = rng.normal(0, 1, n)
    p = _problem_from_dense(A, gens, C, k=n, dt=0.3, steps=6, b=b, center=center)
    res = OT.verify_transposed(p)
    exact = _dense_basis(p, range(7))
    np.testing.assert_allclose(res["basis"], exact, rtol=1e-10, atol=1e-10)
    # and the forward route agrees (both exact)
    fwd = oracle.verify(p, k=n + 1)
    np.testing.assert_allclose(res["basis"], fwd["basis"], rtol=1e-10, atol=1e-10)


def test_diagonal_closed_form():
    # A = diag(d): C e^{At} g = sum_i c_i g_i e^{d_i t}, and the forcing
    # column is sum_i c_i b_i (e^{d_i t} - 1) / d_i.  The unit output row is
    # an eigenvector of A^T: its run breaks down at once and is still exact.
    d = np.array([-3.0, -1.0, -0.5, 0.2, 0.7, -2.2])
    n = d.size
    gens = [W.Generator(W.segments_from_ranges([(0, 3)], 1.0), 0.0, 1.0),
            W.Generator(W.segments_from_ranges([(2, 6)], -0.5), 0.0, 1.0)]
    C = [W.segments_from_ranges([(4, 5)]), W.segments_from_ranges([(0, 6)], 0.5)]
    b = np.array([0.3, 0.0, -1.0, 0.5, 2.0, 0.1])
    center = np.array([1.0, 2.0, 0.0, -1.0, 0.0, 0.5])
    p = _problem_from_dense(np.diag(d), gens, C, k=n, dt=0.25, steps=8, b=b, center=center, symmetric=True)
    res = OT.verify_transposed(p)
    assert res["runs"][0].k_eff == 1
    G = np.stack([g.seg.dense(n) for g in gens] + [center])
    for s in range(9):
        t = s * p.dt
        for q, seg in enumerate(C):
            c = seg.dense(n)
            want = [float(np.sum(c * Gj * np.exp(d * t))) for Gj in G]
            want.append(float(np.sum(c * b * np.expm1(d * t) / d)))
            np.testing.assert_allclose(res["basis"][s, q], want, rtol=1e-12, atol=1e-13)


def test_krylov_error_small_and_shrinking_below_full_dimension():
    # k < n: the transposed approximant converges to the exact basis
    p = W.random_symmetric(n=120, k=6, steps=10, dt=0.05, ngen=3, o=2, affine=True, center=True)
    exact = _dense_basis(p, range(11))
    errs = []
    for k in (6, 12, 24):
        res = OT.verify_transposed(p, k=k)
        errs.append(float(np.abs(res["basis"] - exact).max()))
    scale = float(np.abs(exact).max())
    assert errs[2] < 1e-10 * scale
    assert errs[0] > errs[1] > errs[2] or errs[1] < 1e-12 * scale


def test_forward_and_transposed_agree_at_full_dimension():
    p = W.random_symmetric(n=40, k=40, steps=12, dt=0.05, ngen=3, o=2, affine=True, center=True)
    fwd = oracle.verify(p, k=41)
    tr = OT.verify_transposed(p, k=40)
    assert fwd["roles"] == tr["roles"]
    np.testing.assert_allclose(tr["basis"], fwd["basis"], rtol=1e-9, atol=1e-11)
    assert tr["verdict"]["first_step"] == fwd["verdict"]["first_step"]


def test_one_output_row_one_run():
    # eight initial-space columns, one output: a single simulation
    p = W.heat3d_many_inputs(m=12, k=10, steps=20)
    R, roles = OT.initial_rows(p)
    assert roles == ["gen"] * len(p.gens) + ["center", "affine"]
    assert R.shape == (len(p.gens) + 2, p.n)
    runs, _ = OT.transposed_runs(p)
    assert len(runs) == 1
    assert sp.issparse(R)
