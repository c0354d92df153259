"""The paper-faithful 3D heat system (workloads.heat3d_paper): its matrix
against closed forms.  The cell-centred Laplacian with insulated ends is
diagonalised by the DCT-II, with eigenvalues -4c sin^2(j pi / (2m)),
j = 0..m-1 (a textbook result); the 3D operator is their Kronecker sum, so
without heat exchange the spectrum is every sum of three of them, and the
insulated block conserves heat (A 1 = 0).  The exchange term only lowers the
diagonal of the x = 1 face."""
import itertools
import math

import numpy as np
import scipy.sparse as sp

import workloads as W


def _dense(rowptr, colidx, vals, n):
    return sp.csr_matrix((vals, colidx, rowptr), shape=(n, n)).toarray()


def test_insulated_operator_spectrum_is_the_dct_kronecker_sum():
    m, c = 5, 1.7
    n = m**3
    A = _dense(*W.csr_heat_insulated(m, c, 0.0), n)
    assert np.array_equal(A, A.T)
    assert np.abs(A @ np.ones(n)).max() <= 1e-13 * c
    lam1 = [-4.0 * c * math.sin(j * math.pi / (2 * m)) ** 2 for j in range(m)]
    want = np.sort([a + b + d for a, b, d in itertools.product(lam1, repeat=3)])
    got = np.linalg.eigvalsh(A)
    assert np.abs(got - want).max() <= 1e-12 * 12 * c


def test_exchange_face_and_problem_shape():
    p = W.heat3d_paper(m=6)
    m, c, h = 6, p.meta["c"], p.meta["h"]
    A = _dense(p.rowptr, p.colidx, p.vals, p.n)
    B = _dense(*W.csr_heat_insulated(m, c, 0.0), p.n)
    d = np.diag(A - B)
    ix = np.arange(p.n) // (m * m)
    assert np.allclose(d[ix == m - 1], -c * h * 0.5, rtol=0, atol=1e-15 * c) and np.all(d[ix < m - 1] == 0)
    assert np.array_equal(A - np.diag(np.diag(A)), B - np.diag(np.diag(B)))
    # heat only leaves: A is negative definite with exchange on one face
    assert np.linalg.eigvalsh(A).max() < 0
    # initial region x in [0, 0.4], y in [0, 0.2], z in [0, 0.1]; centre = 8 cells around (0.5, 0.5, 0.5)
    q = W.heat3d_paper(m=20)
    assert q.gens[0].seg.count == 8 * 4 * 2 and q.C[0].count == 8
    assert abs(q.C[0].w.sum() * 1 - q.C[0].nseg * q.C[0].w[0]) == 0.0
    assert (q.steps, q.dt) == (1000, 0.02)


def test_stencil_form_expands_to_the_same_operator():
    m = 7
    p = W.heat3d_paper(m=m)
    s = W.heat3d_paper_stencil(m=m, k=20)
    A = _dense(p.rowptr, p.colidx, p.vals, p.n)
    B = _dense(*s.csr(), s.n)
    assert np.abs(A - B).max() <= 1e-13 * p.meta["c"]
    assert [g.seg.count for g in s.gens] == [g.seg.count for g in p.gens]
    assert np.array_equal(s.C[0].lo, p.C[0].lo) and s.C[0].w[0] == p.C[0].w[0]


def test_paper_norm_at_t50_fixes_the_grid_spacing():
    # Section 4.2 prints |A t| = 32771611 for the 100^3 system at t = 50; the
    # Frobenius norm of 50 A with h = 1 / (m + 1) reproduces it (h = 1 / m
    # would give 32125884, 2 % off)
    p = W.heat3d_paper(m=100)
    fro = 50.0 * math.sqrt(float(np.sum(p.vals * p.vals)))
    assert abs(fro - 32771611.0) <= 1e-7 * 32771611.0
    s = W.heat3d_paper_stencil(m=100)
    assert s.meta["h"] == p.meta["h"] == 1.0 / 101 and s.meta["c"] == p.meta["c"]
