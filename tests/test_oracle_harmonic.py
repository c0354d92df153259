"""The paper's worked example (Section 2.2, Figure 'outline', Section 4.1)
reproduced by the oracle; expected values are the printed ones stored in
tests/golden/harmonic.json."""
import json
import math
import os

import numpy as np
import scipy.linalg
import scipy.sparse as sp

import oracle
import workloads as W

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "harmonic.json")))
TOL = 5e-3   # the paper prints 2-3 significant digits

# the four-variable linear system of Section 2.2 (x, y, t, a)
A4 = np.array([[0.0, 1, 0, 0], [-1, 0, 0, 0], [0, 0, 0, 1], [0, 0, 0, 0]])


def test_augmentation_reproduces_paper_matrix():
    p = W.harmonic_oscillator()
    Aaug = oracle.augment(oracle.system_matrix(p), p.b).toarray()
    np.testing.assert_array_equal(Aaug, A4)


def test_full_basis_at_violation_time():
    t = GOLD["time_of_violation"]
    C = sp.csr_matrix(np.eye(4))
    rows = []
    for i in range(4):
        e = np.zeros(4); e[i] = 1.0
        r = oracle.arnoldi(sp.csr_matrix(A4), e, 4, C)
        rows.append(r.beta0 * r.P @ oracle.expm_pade13(r.H * t)[:, 0])
    full = np.array(rows).T          # column i = e^{At} e_i
    np.testing.assert_allclose(full, GOLD["full_basis_rows_at_3pi_over_4"]["rows"], atol=TOL)


def test_projected_bases_and_transpose_simulation():
    t = GOLD["time_of_violation"]
    A = sp.csr_matrix(A4)
    # transpose simulation from C^T = e_x (Section 4.1)
    e = np.array([1.0, 0, 0, 0])
    r = oracle.arnoldi(A.T.tocsr(), e, 4, sp.csr_matrix(np.eye(4)))
    state = r.beta0 * r.P @ oracle.expm_pade13(r.H * t)[:, 0]
    np.testing.assert_allclose(state, GOLD["transpose_state_at_3pi_over_4"]["state"], atol=TOL)
    np.testing.assert_allclose(state, GOLD["projected_basis_at_3pi_over_4"]["row"], atol=TOL)
    # forward simulation from the paper's two E columns (merged fixed column)
    E = np.array([[0.0, 1, 0, 0], [-5, 0, 0, 1]]).T
    Crow = sp.csr_matrix(np.array([[1.0, 0, 0, 0]]))
    cols = []
    for j in range(2):
        r = oracle.arnoldi(A, E[:, j], 4, Crow)
        cols.append((r.beta0 * r.P @ oracle.expm_pade13(r.H * t)[:, 0])[0])
    np.testing.assert_allclose(cols, GOLD["projected_basis_CeAtE_at_3pi_over_4"]["row"], atol=TOL)
    # transpose route: E^T e^{A^T t} C^T gives the same row
    np.testing.assert_allclose(E.T @ state, cols, atol=1e-12)


def test_split_runs_sum_to_paper_basis():
    # Our split: generator e_y, center (-5,0,0), affine [0;1]; the fixed
    # runs add up to the paper's merged column (-5,0,0,1).
    p = W.harmonic_oscillator()
    res = oracle.verify(p)
    assert res["roles"] == ["gen", "center", "affine"]
    M = res["basis"][3, 0]
    paper = GOLD["projected_basis_CeAtE_at_3pi_over_4"]["row"]
    np.testing.assert_allclose([M[0], M[1] + M[2]], paper, atol=TOL)
    for rr in res["runs"]:
        assert rr.k_eff == 2          # every run terminates exactly


def test_verdicts_and_counter_example():
    p = W.harmonic_oscillator()
    res = oracle.verify(p)
    v = res["verdict"]
    g = GOLD["verdicts"]
    assert v["first_step"] == g["unsafe_first_step"]
    for s in g["safe_steps"]:
        assert not v["unsafe_mask"][s].any()
    ce = GOLD["counter_example"]
    x0 = np.array([-5.0, v["z"][0], 0.0, 1.0])
    np.testing.assert_allclose(x0, ce["x0"], atol=TOL)
    t = v["first_step"] * p.dt
    x = scipy.linalg.expm(A4 * t) @ x0
    np.testing.assert_allclose(x, ce["x"], atol=TOL)
    assert abs(v["y"] - 4.0) < 1e-12
    # the reported output value is the state's x component
    assert abs(x[0] - v["y"]) < 1e-9
