"""Pins of the error-controlled Krylov dimension (oracle/adaptive.py):
the quadrature rule against closed-form integrals, the Lemma 1 bound against
the true error from SciPy's dense expm (plain and augmented runs), exact
breakdown, and the checkpoint schedule of Algorithms 2 and 4."""
import math

import numpy as np
import pytest
import scipy.linalg as sla

import oracle
import workloads as W
from oracle import adaptive as AD


def test_schedule_is_ceil_of_1_1_k():
    got = list(AD.k_schedule(4, 60))
    want, k = [], 4
    while k <= 60:
        want.append(k)
        k = math.ceil(round(1.1 * k, 9))
    assert got == want == [4, 5, 6, 7, 8, 9, 10, 11, 13, 15, 17, 19, 21, 24, 27, 30, 33, 37, 41, 46, 51, 57]


@pytest.mark.parametrize("theta", [-1e4, -3.0, 0.0, 0.5])
def test_quadrature_closed_forms(theta):
    tau = 2.5
    x, w = AD.quadrature_nodes(tau)
    exact = tau if theta == 0.0 else (math.exp(theta * tau) - 1.0) / theta
    assert abs(np.sum(w * np.exp(theta * x)) - exact) <= 1e-13 * max(1.0, abs(exact))
    # weight (tau - t): int_0^tau (tau - t) e^{theta t} dt
    exact2 = tau**2 / 2 if theta == 0.0 else (math.exp(theta * tau) - 1.0 - theta * tau) / theta**2
    assert abs(np.sum(w * (tau - x) * np.exp(theta * x)) - exact2) <= 1e-12 * max(1.0, abs(exact2))


def _true_error(A, v, H, V, beta0, ts):
    e1 = np.zeros(H.shape[0]); e1[0] = 1.0
    return max(np.linalg.norm(sla.expm(A * t) @ v - beta0 * V @ (sla.expm(H * t) @ e1)) for t in ts)


@pytest.mark.parametrize("k", [4, 8, 13, 21])
def test_bound_dominates_true_error(k):
    p = W.small_heat3d(m=8, k=k, steps=50)
    A = oracle.system_matrix(p)
    Ad = A.toarray()
    C = oracle.output_matrix(p)
    v = p.gens[0].seg.dense(p.n)
    r = oracle.arnoldi(A, v, k, C, keep_V=True)
    tau = p.steps * p.dt
    lam = AD.gershgorin_sym_upper(A)
    b = AD.lemma1_bound(r.H, r.h_next, r.beta0, tau, lam)
    err = _true_error(Ad, v, r.H, r.V, r.beta0, np.linspace(0, tau, 26))
    # the bound dominates the true error (up to the rounding of the dense reference)
    assert b >= err - 1e-12 * np.linalg.norm(v)


def test_affine_bound_dominates_true_error():
    p = W.small_heat3d(m=8, k=12, steps=50)
    A = oracle.system_matrix(p)
    Ad = A.toarray()
    C = oracle.output_matrix(p)
    b = p.forcing()
    k = 10
    r = oracle.arnoldi(A, b, k, C, keep_V=True)        # Lanczos space from b, orthonormal
    tau = p.steps * p.dt
    lam = AD.gershgorin_sym_upper(A)
    bound = AD.lemma1_bound(r.H, r.h_next, r.beta0, tau, lam, affine=True)
    # x(t) = A^-1 (e^{At} - I) b against the integral of the Krylov approximation
    e1 = np.zeros(k); e1[0] = 1.0
    worst = 0.0
    for t in np.linspace(0, tau, 21):
        exact = np.linalg.solve(Ad, sla.expm(Ad * t) @ b - b)
        M = np.zeros((k + 1, k + 1)); M[1:, 1:] = r.H; M[1, 0] = 1.0
        approx = r.beta0 * r.V @ sla.expm(M * t)[1:, 0]
        worst = max(worst, np.linalg.norm(exact - approx))
    assert bound >= worst - 1e-12 * np.linalg.norm(b)


def test_breakdown_gives_zero_bound_and_exact_result():
    p = W.heat1d(n=60, k=12, steps=20)
    n = p.n
    x = np.arange(1, n + 1) / (n + 1)
    p.gens = [W.Generator(W.Segments(np.arange(n), np.arange(n) + 1, np.sin(3 * math.pi * x)), 1.0, 0.1)]
    p.C = [W.segments_from_ranges([(10, 30)], 0.05)]
    p.unsafe = np.array([[math.inf, math.inf]])
    res = AD.adaptive_verify(p, eps=1e-6)
    assert res["runs"][0]["k_stop"] == 1 and res["runs"][0]["bound"] == 0.0


def test_adaptive_stops_at_first_checkpoint_under_target():
    p = W.small_heat3d(m=10, k=56, steps=100)
    res = AD.adaptive_verify(p, eps=1e-6)
    A = oracle.system_matrix(p)
    lam = AD.gershgorin_sym_upper(A)
    tau = p.steps * p.dt
    for run, info in zip(oracle.build_runs(p), res["runs"]):
        ks = info["k_stop"]
        assert info["bound"] < 1e-6
        affine = run.role == "affine"
        v = p.forcing() if affine else run.start
        kk = ks
        r = oracle.lanczos(A, v, kk, oracle.output_matrix(p), opnorm=oracle.krylov.inf_norm(A))
        assert abs(AD.lemma1_bound(r.H, r.h_next, r.beta0, tau, lam, affine) - info["bound"]) <= 1e-9 * info["bound"]
        earlier = [c for c in AD.k_schedule(4, ks) if c < ks]
        if earlier:
            c = earlier[-1]
            r2 = oracle.lanczos(A, v, c, oracle.output_matrix(p), opnorm=oracle.krylov.inf_norm(A))
            assert AD.lemma1_bound(r2.H, r2.h_next, r2.beta0, tau, lam, affine) >= 1e-6
