"""Pins of the oracle's Krylov processes and the whole projected path:
Arnoldi/Lanczos invariants, exact termination (breakdown) cases with closed
forms, brute-force dense exponentials, and the exact 3D heat solution by a
separable sine transform including the affine term."""
import math

import numpy as np
import pytest
import scipy.linalg
import scipy.sparse as sp

import oracle
from oracle.krylov import Run, build_runs, krylov_run
import workloads as W


def _rand_sym(n, seed):
    rng = np.random.default_rng(seed)
    M = sp.random(n, n, density=6.0 / n, random_state=seed, data_rvs=lambda s: rng.normal(size=s))
    M = (M + M.T) * 0.5
    d = np.abs(M).sum(axis=1).A1 + 1.0
    return (M - sp.diags(d)).tocsr()


def test_arnoldi_relation_and_orthogonality():
    rng = np.random.default_rng(0)
    n, k = 120, 25
    A = sp.csr_matrix(rng.normal(size=(n, n)) / math.sqrt(n))
    C = sp.csr_matrix(rng.normal(size=(2, n)))
    v = rng.normal(size=n)
    r = oracle.arnoldi(A, v, k, C, keep_V=True)
    V, H = r.V, r.H
    assert r.k_eff == k
    np.testing.assert_allclose(V.T @ V, np.eye(k), atol=1e-14)
    # A V_k = V_k H_k + h_{k+1,k} v_{k+1} e_k^T; the residual is orthogonal to V_k
    R = A @ V - V @ H
    np.testing.assert_allclose(R[:, :-1], 0.0, atol=1e-13)
    assert abs(np.linalg.norm(R[:, -1]) - r.h_next) <= 1e-12 * r.h_next
    np.testing.assert_allclose(V.T @ R[:, -1], 0.0, atol=1e-13)
    np.testing.assert_allclose(r.P, C @ V, atol=1e-14)
    assert abs(r.beta0 - np.linalg.norm(v)) <= 1e-14 * r.beta0
    assert np.all(np.tril(H, -2) == 0.0)           # upper Hessenberg


def test_lanczos_is_tridiagonal_and_matches_arnoldi_on_symmetric():
    n, k = 200, 30
    A = _rand_sym(n, 1)
    rng = np.random.default_rng(1)
    C = sp.csr_matrix(rng.normal(size=(3, n)))
    v = rng.normal(size=n)
    L = oracle.lanczos(A, v, k, C)
    R = oracle.arnoldi(A, v, k, C, keep_V=True)
    assert L.k_eff == R.k_eff == k
    T = L.H
    assert np.all(np.triu(T, 2) == 0.0) and np.all(np.tril(T, -2) == 0.0)
    np.testing.assert_array_equal(T, T.T)
    # the two processes differ only by rounding on a well-conditioned start
    np.testing.assert_allclose(T, R.H, atol=1e-10 * np.abs(T).max())
    np.testing.assert_allclose(L.P, R.P, atol=1e-10 * np.abs(R.P).max())
    # Lanczos H equals V^T A V of the (orthonormal) Arnoldi basis
    np.testing.assert_allclose(T, R.V.T @ (A @ R.V), atol=1e-10 * np.abs(T).max())


def test_diagonal_terminates_exactly():
    # A with 4 distinct eigenvalues: the Krylov space is invariant at k=4
    lam = np.array([-3.0, -0.5, -0.5, -1.25, -3.0, -0.1, -1.25])
    A = sp.diags(lam).tocsr()
    v = np.arange(1.0, 8.0)
    C = sp.csr_matrix(np.eye(7))
    for proc in (oracle.lanczos, oracle.arnoldi):
        r = proc(A, v, 10, C)
        assert r.k_eff == 4
        for t in (0.0, 0.3, 2.0):
            y = r.beta0 * r.P @ (oracle.expm_pade13(r.H * t)[:, 0])
            np.testing.assert_allclose(y, np.exp(lam * t) * v, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("mode", [1, 3, 7])
def test_heat1d_sine_mode_breaks_down_at_k1(mode):
    # Dirichlet 1D heat: sin(j pi x_i) is an eigenvector with
    # lambda_j = -(4/h^2) sin^2(j pi h / 2)
    p = W.heat1d()
    A = oracle.system_matrix(p)
    n = p.n
    h = 1.0 / (n + 1)
    x = np.arange(1, n + 1) * h
    v = np.sin(mode * math.pi * x)
    lam = -(4.0 / h**2) * math.sin(mode * math.pi * h / 2) ** 2
    C = oracle.output_matrix(p)
    r = oracle.lanczos(A, v, 30, C)
    assert r.k_eff == 1
    assert abs(r.H[0, 0] - lam) <= 1e-12 * abs(lam)
    for t in (1e-4, 1e-2):
        y = r.beta0 * r.P @ oracle.expm_pade13(r.H * t)[:, 0]
        np.testing.assert_allclose(y, math.exp(lam * t) * (C @ v), rtol=1e-12)


def test_nilpotent_shift_gives_polynomial():
    # A = down-shift: A e_i = e_{i+1}; e^{At} e_1 = sum_j t^j/j! e_{j+1}
    n = 6
    A = sp.csr_matrix(np.diag(np.ones(n - 1), -1))
    C = sp.csr_matrix(np.eye(n))
    v = np.zeros(n); v[0] = 1.0
    r = oracle.arnoldi(A, v, 10, C)
    assert r.k_eff == n
    t = 1.7
    y = r.beta0 * r.P @ oracle.expm_pade13(r.H * t)[:, 0]
    exact = np.array([t**j / math.factorial(j) for j in range(n)])
    np.testing.assert_allclose(y, exact, rtol=1e-13)


def test_full_krylov_equals_dense_expm():
    # brute force: at k = n the approximant is exact
    n = 60
    A = _rand_sym(n, 5)
    rng = np.random.default_rng(5)
    C = sp.csr_matrix(rng.normal(size=(2, n)))
    v = rng.normal(size=n)
    r = oracle.arnoldi(A, v, n, C)
    Ad = A.toarray()
    for t in (0.01, 0.3, 1.5):
        y = r.beta0 * r.P @ oracle.expm_pade13(r.H * t)[:, 0]
        ref = C @ (scipy.linalg.expm(Ad * t) @ v)
        np.testing.assert_allclose(y, ref, rtol=1e-11, atol=1e-12 * np.abs(ref).max())


def test_augmented_run_closed_form():
    # e^{At}[0;1] top block = A^{-1}(e^{At} - I) b for invertible A
    n = 40
    A = _rand_sym(n, 9)
    rng = np.random.default_rng(9)
    b = rng.normal(size=n)
    Aaug = oracle.augment(A, b)
    assert Aaug.shape == (n + 1, n + 1)
    np.testing.assert_array_equal(Aaug[n].toarray(), 0.0)
    np.testing.assert_array_equal(Aaug[:n, n].toarray().ravel(), b)
    C = sp.csr_matrix(np.hstack([np.eye(n), np.zeros((n, 1))]))
    e = np.zeros(n + 1); e[n] = 1.0
    r = oracle.arnoldi(Aaug, e, n + 1, C)
    Ad = A.toarray()
    for t in (0.05, 0.7, 4.0):
        y = r.beta0 * r.P @ oracle.expm_pade13(r.H * t)[:, 0]
        ref = np.linalg.solve(Ad, (scipy.linalg.expm(Ad * t) - np.eye(n)) @ b)
        np.testing.assert_allclose(y, ref, rtol=1e-10, atol=1e-12 * np.abs(ref).max())
    # the augmented Hessenberg is bordered: first row zero, h21 = |b|
    assert np.all(r.H[0] == 0.0)
    assert abs(r.H[1, 0] - np.linalg.norm(b)) <= 1e-14 * np.linalg.norm(b)


def _dst_truth(m, D, coef_b, gen_vec, C, times):
    """Exact C e^{At} g and C int_0^t e^{A s} b ds for the Dirichlet 3D heat
    operator via its separable sine eigenbasis."""
    h = 1.0 / (m + 1)
    j = np.arange(1, m + 1)
    S = np.sqrt(2.0 / (m + 1)) * np.sin(np.outer(j, j) * math.pi * h)     # orthonormal DST-I
    lam1 = -(4.0 * D / h**2) * np.sin(j * math.pi * h / 2) ** 2
    lam = lam1[:, None, None] + lam1[None, :, None] + lam1[None, None, :]

    def fwd(v):
        X = v.reshape(m, m, m)
        return np.einsum("ai,bj,ck,ijk->abc", S, S, S, X)

    def inv(Y):
        return np.einsum("ai,bj,ck,abc->ijk", S, S, S, Y).ravel()

    gh, bh = fwd(gen_vec), fwd(coef_b)
    out_g, out_b = [], []
    for t in times:
        out_g.append(C @ inv(np.exp(lam * t) * gh))
        out_b.append(C @ inv(np.expm1(lam * t) / lam * bh))
    return np.array(out_g), np.array(out_b)


def test_heat3d_pipeline_against_sine_transform_truth():
    # small m so that the Krylov space is (numerically) converged at k=n/2
    p = W.small_heat3d(m=6, k=60, steps=6, dt=0.5)
    res = oracle.verify(p)
    assert res["roles"] == ["gen", "affine"]
    C = oracle.output_matrix(p)
    times = np.arange(p.steps + 1) * p.dt
    g = p.gens[0].seg.dense(p.n)
    yg, yb = _dst_truth(6, 0.01, p.b, g, C, times)
    scale = np.abs(yg).max()
    np.testing.assert_allclose(res["basis"][:, :, 0], yg, atol=1e-10 * scale)
    np.testing.assert_allclose(res["basis"][:, :, 1], yb, atol=1e-10 * np.abs(yb).max())


def test_heat3d_lanczos_lemma_free_convergence_is_monotone():
    # |e^{At} v| is non-increasing for symmetric negative definite A; the
    # converged Krylov state inherits it.
    p = W.small_heat3d(m=5, k=60, steps=8, dt=0.3)
    A = oracle.system_matrix(p)
    I = sp.identity(p.n, format="csr")
    r = oracle.lanczos(A, p.gens[0].seg.dense(p.n), 60, I)
    norms = [np.linalg.norm(r.beta0 * r.P @ oracle.expm_pade13(r.H * s * p.dt)[:, 0])
             for s in range(p.steps + 1)]
    assert all(b <= a * (1 + 1e-12) for a, b in zip(norms, norms[1:]))


def test_runs_split_and_roles():
    p = W.random_symmetric(affine=True, center=True, ngen=3)
    runs = build_runs(p)
    assert [r.role for r in runs] == ["gen", "gen", "gen", "center", "affine"]
    assert runs[-1].start.size == p.n + 1 and runs[-1].start[-1] == 1.0
    # basis at step 0 is C E exactly (up to rounding in beta0 * (C v / beta0))
    res = oracle.verify(p, steps=3)
    C = oracle.output_matrix(p)
    for i, r in enumerate(runs[:-1]):
        np.testing.assert_allclose(res["basis"][0, :, i], C @ r.start, rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(res["basis"][0, :, -1], 0.0, atol=1e-15)


def test_zero_generator_contributes_zero():
    p = W.random_symmetric(affine=False, ngen=2)
    p.gens[1].seg.w[:] = 0.0
    res = oracle.verify(p, steps=2)
    assert res["runs"][1].k_eff == 0
    assert np.all(res["basis"][:, :, 1] == 0.0)


def test_structural_zero_outputs_are_exact():
    # 1D heat, k=30 from x_1..x_10 never reaches x_90..x_110
    p = W.heat1d(steps=20)
    res = oracle.verify(p)
    assert np.all(res["basis"] == 0.0)
    assert res["verdict"]["first_step"] == -1
