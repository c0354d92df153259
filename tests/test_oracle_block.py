"""Pins of the block Arnoldi oracle (oracle/block.py) against facts that do
not come from it: the single-vector Arnoldi of Algorithm 1 (p = 1), the block
Arnoldi relation and orthonormality, SciPy's dense expm when the block space
is the whole space, column-permutation invariance of the approximant, and
exact eigenvector blocks."""
import math

import numpy as np
import pytest
import scipy.linalg as sla

import oracle
import workloads as W
from oracle import block as OB


def _conv(nx=6, ny=5, nz=7, seed=3, gen_len=6):
    p = W.conv_diff3d(nx, ny, nz, ngen=4, gen_len=gen_len, o=3, k=6, steps=20, dt=2e-3, seed=seed)
    return p, oracle.system_matrix(p), oracle.output_matrix(p)


def _G(p, cols=None):
    gens = p.gens if cols is None else [p.gens[c] for c in cols]
    return np.stack([g.seg.dense(p.n) for g in gens], axis=1)


def test_p1_reduces_to_arnoldi():
    p, A, C = _conv()
    g = _G(p, [0])
    blk = OB.block_arnoldi(A, g, 8, C)
    ref = oracle.arnoldi(A, g[:, 0], 8, C)
    assert blk.k_eff == ref.k_eff
    np.testing.assert_allclose(blk.R0[0, 0], ref.beta0, rtol=1e-14)
    np.testing.assert_allclose(blk.H, ref.H, rtol=0, atol=1e-12 * np.abs(ref.H).max())
    np.testing.assert_allclose(blk.P, ref.P, rtol=0, atol=1e-12 * np.abs(ref.P).max())


def test_block_arnoldi_relation_and_orthonormality():
    p, A, C = _conv()
    G = _G(p)
    k = 5
    blk = OB.block_arnoldi(A, G, k, C, keep_V=True)
    V = blk.V
    m = V.shape[1]
    np.testing.assert_allclose(V.T @ V, np.eye(m), atol=1e-13)
    # A V_k - V_k H_k is supported on the last block column, where it equals
    # the next block times h_next; its columns are orthogonal to V_k
    Rres = A @ V - V @ blk.H
    np.testing.assert_allclose(Rres[:, :m - blk.p], 0.0, atol=1e-11 * np.abs(A).max())
    last = Rres[:, m - blk.p:]
    np.testing.assert_allclose(V.T @ last, 0.0, atol=1e-11 * np.abs(A).max())
    np.testing.assert_allclose(np.linalg.norm(last, axis=0), np.linalg.norm(blk.h_next, axis=0), rtol=1e-10)
    # G = V_1 R0 with R0 upper triangular, non-negative diagonal
    np.testing.assert_allclose(V[:, :blk.p] @ blk.R0, G, atol=1e-13 * np.abs(G).max())
    assert np.allclose(np.tril(blk.R0, -1), 0.0) and np.all(np.diag(blk.R0) >= 0)


def test_full_space_equals_dense_expm():
    # p k >= n: the block space is all of R^n and the approximant is exact
    p, A, C = _conv(nx=3, ny=3, nz=4, gen_len=3)
    G = _G(p)
    n = p.n
    k = math.ceil(n / G.shape[1]) + 1
    blk = OB.block_arnoldi(A, G, k, C)
    Ad = A.toarray()
    Cd = C.toarray()
    for t in (0.0, 0.01, 0.05, 0.3):
        want = Cd @ sla.expm(Ad * t) @ G
        E = sla.expm(blk.H * t)
        got = blk.P @ (E[:, :blk.p] @ blk.R0)
        np.testing.assert_allclose(got, want, rtol=0, atol=1e-11 * max(1.0, np.abs(want).max()))


def test_column_permutation_invariance():
    # the block Krylov space does not depend on the order of G's columns
    p, A, C = _conv()
    perm = [2, 0, 3, 1]
    a = OB.block_arnoldi(A, _G(p), 4, C)
    b = OB.block_arnoldi(A, _G(p, perm), 4, C)
    for t in (0.01, 0.1):
        ya = a.P @ (sla.expm(a.H * t)[:, :a.p] @ a.R0)
        yb = b.P @ (sla.expm(b.H * t)[:, :b.p] @ b.R0)
        np.testing.assert_allclose(yb, ya[:, perm], rtol=0, atol=1e-12 * np.abs(ya).max())


def test_eigenvector_block_breaks_down_exactly():
    # two Dirichlet sine modes of the 1D heat matrix span an invariant space
    hp = W.heat1d(n=60, k=5, steps=10)
    hp.C = [W.segments_from_ranges([(20, 40)], 0.05)]
    A = oracle.system_matrix(hp)
    C = oracle.output_matrix(hp)
    n = hp.n
    x = np.arange(1, n + 1) / (n + 1)
    G = np.stack([np.sin(2 * math.pi * x), np.sin(5 * math.pi * x)], axis=1)
    blk = OB.block_arnoldi(A, G, 5, C)
    assert blk.k_eff == 1
    lam = np.array([-4 * (n + 1) ** 2 * math.sin(j * math.pi / (2 * (n + 1))) ** 2 for j in (2, 5)])
    t = 3e-4
    want = C.toarray() @ (G * np.exp(lam * t)[None, :])
    got = blk.P @ (sla.expm(blk.H * t)[:, :2] @ blk.R0)
    np.testing.assert_allclose(got, want, rtol=1e-10, atol=1e-14)


def test_rank_deficient_start_is_rejected():
    p, A, C = _conv()
    G = _G(p, [0, 0])
    with pytest.raises(ValueError):
        OB.block_arnoldi(A, G, 3, C)


def test_block_verify_matches_column_results():
    # the basis columns of block_verify are the per-block approximants
    p = W.conv_diff3d(5, 5, 6, ngen=5, gen_len=5, o=2, k=4, steps=6, dt=1e-3, seed=9)
    res = OB.block_verify(p, p=3)
    assert res["basis"].shape == (7, 2, 5)
    A, C = oracle.system_matrix(p), oracle.output_matrix(p)
    second = OB.block_arnoldi(A, _G(p, [3, 4]), 4, C)
    want = OB.block_project_steps(second, p.dt, p.steps)
    np.testing.assert_array_equal(res["basis"][:, :, 3:5], want)
    assert res["verdict"]["first_step"] >= -1
