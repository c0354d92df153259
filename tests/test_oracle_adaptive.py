"""Pins of the error-controlled Krylov dimension (oracle/adaptive.py):
the quadrature rule against closed-form integrals; the Lemma 1 bound against
a one-step case worked by hand with lambda_max > 0 (both sides of the bound,
the factor e^{lambda tau} and the Gershgorin bound), against the true error
from SciPy's dense expm (plain and augmented runs) and against the paper's
own result on its 100^3 heat system (Section 5.3: the bound first drops
below 1e-6 at k = 544, at 5.8e-7); exact breakdown; and the checkpoint
schedule of Algorithms 2 and 4."""
import math
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import oracle
import workloads as W
from oracle import adaptive as AD


def test_schedule_is_ceil_of_the_double_product():
    # ceil(1.1 k) with 1.1 k rounded to the nearest double: the exact product
    # of k and the double nearest 1.1, rounded once (Fraction -> float rounds
    # correctly), then the ceiling
    got = list(AD.k_schedule(4, 700))
    want, k = [], 4
    while k <= 700:
        want.append(k)
        k = math.ceil(float(Fraction(1.1) * k))
    assert got == want
    # the double product first exceeds an integer at 1.1 * 170 = 187.00000000000003
    assert got[got.index(170) + 1] == 188
    # Section 5.3 reports a stop at k = 544: it lies on this sequence, the
    # exact-arithmetic ceiling (..., 491, 541, 596) would not reach it
    assert [494, 544, 599] == got[got.index(494):got.index(494) + 3]
    exact, k = [], 4
    while k <= 700:
        exact.append(k)
        k = (11 * k + 9) // 10
    assert 544 not in exact


def test_one_step_bound_by_hand_with_positive_lambda():
    # A = diag(1, 1/2), v = (1, 1) (normalised by the process).  One Lanczos
    # step: alpha = 3/4, the residual ((1 - 3/4), (1/2 - 3/4)) / sqrt 2 has
    # norm beta = 1/4.  lambda_max = 1 > 0, so Lemma 1 gives
    #   bound(tau) = (1/4) e^{tau} int_0^tau e^{3t/4} dt = (1/4) e^tau (e^{3 tau/4} - 1) / (3/4).
    A = np.diag([1.0, 0.5])
    C = np.eye(2)
    tau = 2.0
    lam = AD.gershgorin_sym_upper(A)
    assert lam == 1.0
    r = AD.adaptive_lanczos(A, np.array([1.0, 1.0]), C, 0.0, tau, 1, lam, 1.0)
    assert r["k_stop"] == 1 and abs(r["H"][0, 0] - 0.75) <= 1e-15 and abs(r["h"] - 0.25) <= 1e-15
    want = 0.25 * math.exp(tau) * (math.exp(0.75 * tau) - 1.0) / 0.75
    got = AD.lemma1_bound(r["H"], r["h"], tau, lam)
    assert abs(got - want) <= 1e-13 * want
    # and the bound holds: |e^{tA} v - e^{t alpha} v| for unit v at every t <= tau
    for t in np.linspace(0.0, tau, 9):
        err = math.hypot(math.exp(t) - math.exp(0.75 * t), math.exp(0.5 * t) - math.exp(0.75 * t)) / math.sqrt(2)
        assert err <= AD.lemma1_bound(r["H"], r["h"], t, lam) + 1e-15
    # the augmented weight (tau - t): (1/4) e^tau int_0^tau (tau - t) e^{3t/4} dt
    want_aff = 0.25 * math.exp(tau) * (math.exp(0.75 * tau) - 1.0 - 0.75 * tau) / 0.75**2
    assert abs(AD.lemma1_bound(r["H"], r["h"], tau, lam, affine=True) - want_aff) <= 1e-13 * want_aff
    # a nonpositive lambda contributes a factor 1
    assert abs(AD.lemma1_bound(r["H"], r["h"], tau, -3.0) - want * math.exp(-tau)) <= 1e-13 * want


def test_gershgorin_bound_by_hand():
    # [[0.2, 0.7], [-0.1, 1.0]]: the off-diagonal of the symmetric part,
    # |0.7 - 0.1| / 2 = 0.3, is taken as at most (0.7 + 0.1) / 2 = 0.4: row
    # bounds 0.2 + 0.4 and 1.0 + 0.4 (the symmetric part's eigenvalues are
    # 0.6 +- 0.5, so 1.4 >= 1.1 holds)
    A = np.array([[0.2, 0.7], [-0.1, 1.0]])
    assert abs(AD.gershgorin_sym_upper(A) - 1.4) <= 1e-15
    assert AD.gershgorin_sym_upper(A) >= np.linalg.eigvalsh(0.5 * (A + A.T)).max()
    # same-sign mirrored entries lose nothing: [[0, 0.7], [0.1, 0]] -> 0.4,
    # the largest eigenvalue of its symmetric part
    A2 = np.array([[0.0, 0.7], [0.1, 0.0]])
    assert abs(AD.gershgorin_sym_upper(A2) - 0.4) <= 1e-15
    # one-sided entries count half in their row and half in their column
    A3 = np.array([[0.0, 1.0, 0.0], [0.0, 0.0, 0.0], [0.0, 0.0, -1.0]])
    assert AD.gershgorin_sym_upper(A3) == 0.5
    # negative off-diagonals count by magnitude
    B = np.array([[-2.0, -0.5, 0.0], [-0.5, -1.0, 0.25], [0.0, 0.25, 0.1]])
    assert abs(AD.gershgorin_sym_upper(B) - 0.35) <= 1e-15


def test_symmetric_route_equals_pade_route():
    # (e^{tT})_{k,1} through the eigen-decomposition of a symmetric
    # tridiagonal T against the Pade exponential of the same matrix
    p = W.small_heat3d(m=8, k=15, steps=50)
    A = oracle.system_matrix(p)
    r = oracle.lanczos(A, p.gens[0].seg.dense(p.n), 15, oracle.output_matrix(p))
    assert AD.is_sym_tridiagonal(r.H)
    ts = np.array([1e-3, 0.1, 0.5, 1.0, 3.0])
    got = AD.h_values(r.H, ts)
    want = np.array([AD.h_entry(r.H, t) for t in ts])
    # the eigen form sums k terms of size <= 1 (|Q| <= 1, theta <= 0): its
    # error is absolute, a few k eps, where the Pade form keeps tiny values
    assert np.abs(got - want).max() <= 4 * 15 * np.finfo(float).eps
    assert abs(got[-1] - want[-1]) <= 1e-9 * abs(want[-1])


@pytest.mark.slow
def test_paper_heat_100_stops_at_k_544():
    # Section 5.3: on the 100^3 heat system the bound first falls below the
    # 1e-6 target at k = 544, where it is 5.8e-7; the checkpoint before (494)
    # must not pass.  One Lanczos run of 544 steps on n = 10^6.
    p = W.heat3d_paper(m=100)
    A = oracle.system_matrix(p)
    lam = AD.gershgorin_sym_upper(A)
    assert lam <= 1e-9 * p.meta["c"]       # insulated + exchange: no growth, factor 1
    v = p.gens[0].seg.dense(p.n)
    r = AD.adaptive_lanczos(A, v, oracle.output_matrix(p), 1e-6, 20.0, 600, lam, oracle.krylov.inf_norm(A))
    assert r["k_stop"] == 544
    assert abs(r["bound"] - 5.8e-7) <= 0.05 * 5.8e-7
    b494 = AD.lemma1_bound(r["H"][:494, :494], r["H"][494, 493], 20.0, lam)
    assert b494 > 1e-6


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
    b = r.beta0 * AD.lemma1_bound(r.H, r.h_next, tau, lam)
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
    bound = r.beta0 * AD.lemma1_bound(r.H, r.h_next, tau, lam, affine=True)
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
        assert abs(AD.lemma1_bound(r.H, r.h_next, tau, lam, affine) - info["bound"]) <= 1e-9 * info["bound"]
        earlier = [c for c in AD.k_schedule(4, ks) if c < ks]
        if earlier:
            c = earlier[-1]
            r2 = oracle.lanczos(A, v, c, oracle.output_matrix(p), opnorm=oracle.krylov.inf_norm(A))
            assert AD.lemma1_bound(r2.H, r2.h_next, tau, lam, affine) >= 1e-6


# ---------------------------------------------------------------------------
# Algorithm 2: the same control around Arnoldi for a general A
# ---------------------------------------------------------------------------

def _shift(n):
    # e_i -> e_{i+1}: Arnoldi from e_1 keeps V = I and H_j = the j x j shift,
    # so (e^{t H_j})_{j,1} = t^{j-1} / (j-1)! and h_{j+1,j} = 1
    return sp.diags([np.ones(n - 1)], [-1], format="csr")


def test_arnoldi_bound_on_a_shift_is_the_taylor_tail():
    n = 40
    A = _shift(n)
    lam = AD.gershgorin_sym_upper(A)
    assert lam == 1.0                    # off-diagonal 1/2 on both sides of interior rows
    C = sp.csr_matrix(np.ones((1, n)))
    tau = 1.0
    v = np.zeros(n); v[0] = 1.0
    # bound(j) = e^tau tau^j / j!: e / 9! = 7.5e-6 > 1e-6 > e / 10! = 7.5e-7,
    # and 10 is a checkpoint (4, 5, ..., 11, 13, ...)
    r = AD.adaptive_arnoldi(A, v, C, 1e-6, tau, 30, lam, 1.0)
    assert r["k_stop"] == 10
    assert abs(r["bound"] - math.e / math.factorial(10)) <= 1e-12 * r["bound"]
    assert r["h"] == 1.0 and np.array_equal(r["H"], np.eye(10, k=-1))
    # the augmented weight: int_0^tau (tau - t) t^{j-1}/(j-1)! dt = tau^{j+1}/(j+1)!
    ra = AD.adaptive_arnoldi(A, v, C, 1e-6, 2.0, 30, lam, 1.0, affine=True)
    j = ra["k_stop"]
    want = math.exp(2.0) * 2.0 ** (j + 1) / math.factorial(j + 1)
    assert abs(ra["bound"] - want) <= 1e-12 * want and want < 1e-6
    prev = [c for c in AD.k_schedule(4, j) if c < j][-1]
    assert math.exp(2.0) * 2.0 ** (prev + 1) / math.factorial(prev + 1) >= 1e-6
    # the true error is the tail of the exponential series: below the bound
    err = math.sqrt(sum((tau**i / math.factorial(i)) ** 2 for i in range(10, 60)))
    assert err <= r["bound"]


def test_arnoldi_breakdown_ends_exactly():
    n = 12
    A = _shift(n)
    v = np.zeros(n); v[0] = 1.0
    C = sp.csr_matrix(np.ones((1, n)))
    # A^12 e_1 = 0: the space is invariant at k = 12, before any checkpoint passes
    r = AD.adaptive_arnoldi(A, v, C, 1e-300, 1.0, 40, 1.0, 1.0)
    assert r["k_stop"] == 12 and r["bound"] == 0.0
    # a zero start vector contributes nothing
    z = AD.adaptive_arnoldi(A, np.zeros(n), C, 1e-6, 1.0, 40, 1.0, 1.0)
    assert z["k_stop"] == 0 and z["bound"] == 0.0


def test_arnoldi_control_equals_lanczos_control_on_a_symmetric_system():
    # the Hessenberg (Pade) route of the integrand against the tridiagonal
    # eigen route, and Arnoldi's H against Lanczos' T, through the whole
    # control: same stops, bounds to rounding, same basis
    p = W.small_heat3d(m=8, k=40, steps=60)
    lz = AD.adaptive_verify(p, eps=1e-7, method="lanczos")
    ar = AD.adaptive_verify(p, eps=1e-7, method="arnoldi")
    for a, b in zip(lz["runs"], ar["runs"]):
        assert a["k_stop"] == b["k_stop"]
        assert abs(a["bound"] - b["bound"]) <= 1e-6 * a["bound"]
    scale = np.abs(lz["basis"]).max()
    assert np.abs(lz["basis"] - ar["basis"]).max() <= 1e-10 * scale


def test_arnoldi_bound_dominates_true_error_nonsymmetric():
    # 6^3 convection-diffusion with off-stencil entries: at the stop the
    # bound exceeds the true error of the normalised process at every
    # t <= tau (the bound grows with tau); also for the augmented run
    p = W.conv_diff3d(6, 6, 6, ngen=2, gen_len=20, o=2, k=40, steps=50, dt=2e-3)
    A = oracle.system_matrix(p)
    Ad = A.toarray()
    C = oracle.output_matrix(p)
    lam = AD.gershgorin_sym_upper(A)
    tau = p.steps * p.dt
    opnorm = oracle.krylov.inf_norm(A)
    for g in p.gens:
        v = g.seg.dense(p.n)
        r = AD.adaptive_arnoldi(A, v, C, 1e-8, tau, 40, lam, opnorm)
        j = r["k_stop"]
        assert 4 <= j < 40 and r["bound"] < 1e-8
        full = oracle.arnoldi(A, v, j, C, keep_V=True)
        assert np.array_equal(full.H, r["H"])
        err = _true_error(Ad, v / r["beta0"], r["H"], full.V, 1.0, np.linspace(0, tau, 11))
        assert err <= r["bound"] + 1e-13
        # one checkpoint earlier the bound was not yet below the target
        prev = [c for c in AD.k_schedule(4, j) if c < j]
        if prev:
            assert AD.lemma1_bound(r["H"][:prev[-1], :prev[-1]], r["H"][prev[-1], prev[-1] - 1], tau, lam) >= 1e-8
    # augmented run from b: x(t) = int_0^t e^{As} b ds against the bordered approximation
    b = np.linspace(-1.0, 1.0, p.n)
    r = AD.adaptive_arnoldi(A, b, C, 1e-9, tau, 39, lam, opnorm, affine=True)
    j = r["k_stop"]
    full = oracle.arnoldi(A, b, j, C, keep_V=True)
    worst = 0.0
    for t in np.linspace(0, tau, 11):
        exact = np.linalg.solve(Ad, sla.expm(Ad * t) @ b - b)
        M = np.zeros((j + 1, j + 1)); M[1:, 1:] = r["H"]; M[1, 0] = 1.0
        approx = r["beta0"] * full.V @ sla.expm(M * t)[1:, 0]
        worst = max(worst, np.linalg.norm(exact - approx))
    assert worst <= r["beta0"] * r["bound"] + 1e-12 * np.linalg.norm(b)


def test_adaptive_verify_nonsymmetric_takes_arnoldi():
    p = W.conv_diff3d(6, 6, 6, ngen=2, gen_len=20, o=2, k=30, steps=40, dt=2e-3)
    res = AD.adaptive_verify(p, eps=1e-7)
    ref = oracle.verify(p, method="arnoldi", k=max(r["k_stop"] for r in res["runs"]))
    for i, info in enumerate(res["runs"]):
        assert 4 <= info["k_stop"] < 30 and info["bound"] < 1e-7
        # the columns equal fixed-k Arnoldi at the stop
        one = oracle.verify(p, method="arnoldi", k=info["k_stop"])
        np.testing.assert_allclose(res["basis"][:, :, i], one["basis"][:, :, i], rtol=0,
                                   atol=1e-12 * np.abs(one["basis"][:, :, i]).max())
    assert res["verdict"]["first_step"] == ref["verdict"]["first_step"]
    with pytest.raises(ValueError):
        AD.adaptive_verify(p, eps=1e-7, method="lanczos")
