"""A-posteriori error control of the Krylov dimension (paper Section 4.2,
Lemma 1 and the red lines of Algorithms 2 and 4): test infrastructure only
(see the package docstring).

Lemma 1 (for e^{-tau B} v, |v| = 1, Arnoldi of B): the error is at most
h_{k+1,k} e^{-min(nu(B), 0) tau} * integral_0^tau |e_k^T e^{-t H^B_k} e_1| dt,
nu(B) the smallest eigenvalue of (B + B^T)/2.  The paper feeds B = -A to get
e^{tau A} v.  Arnoldi of -A has the same vectors as Arnoldi of A up to signs,
so |e_k^T e^{-t H^B_k} e_1| = |(e^{t H_k})_{k,1}| with H_k from A itself, and
-nu(-A) = lambda_max((A + A^T)/2).  Algorithms 2 and 4 take a normalised
start vector and compute-error sees H only, so the bound is that of the
normalised process (an error relative to |v|):

    bound(tau) = h_{k+1,k} e^{max(lambda, 0) tau} int_0^tau |(e^{t H_k})_{k,1}| dt,

lambda any upper bound of lambda_max((A + A^T)/2) (a Gershgorin bound here).

The augmented run approximates x(t) = int_0^t e^{As} b ds by integrating the
Lanczos approximation of e^{As} b (the bordered Krylov matrix does exactly
that), so its error relative to |b| is at most int_0^tau bound_b(s) ds
    = h e^{max(lambda,0) tau} int_0^tau (tau - t) |(e^{t T})_{k,1}| dt
with T and h from the Lanczos process started at b / |b|.

The integral is evaluated by one fixed rule, the definition both sides
implement: composite 8-point Gauss-Legendre on [0, tau 2^-L] and on each
[tau 2^-(i+1), tau 2^-i], i = 0..L-1, every interval split into U equal
parts (L = 40, U = 8).  The geometric intervals resolve the fast transient
of h near t = 0 that a uniform grid misses.  The integrand is the (k, 1)
entry of a Pade exponential of t H_k; for a symmetric tridiagonal H_k (a
Lanczos matrix) it is the same entry written through the eigen-decomposition
H_k = Q diag(theta) Q^T, sum_i Q_{k,i} Q_{1,i} e^{theta_i t}, which makes
Krylov dimensions in the hundreds affordable.

The Krylov dimension is chosen as in Algorithms 2 and 4: check at k = 4,
then k <- ceil(1.1 k), evaluated in IEEE double as printed (1.1 * 170 rounds
to 187.00000000000003, so 170 is followed by 188), stop at the first k whose
bound is below the target.  This is the sequence on which the paper's
Section 5.3 reports its stop at k = 544.

Algorithm 2 is the same control around Arnoldi (Algorithm 1) for a general
A: H_k is then upper Hessenberg and the integrand takes the Pade route.
Arnoldi's first j columns do not depend on the later ones, so the bound at
checkpoint j is that of the leading j x j block of one run to the cap, with
h_{j+1,j} its next sub-diagonal entry.
"""
from __future__ import annotations

import math

import numpy as np

import scipy.linalg as sla

from .krylov import BREAKDOWN_FACTOR, EPS, _breaks_down, arnoldi, expm_pade13

QUAD_LEVELS = 40
QUAD_SPLIT = 8
GL_NODES, GL_WEIGHTS = np.polynomial.legendre.leggauss(8)


def quadrature_nodes(tau: float):
    """Nodes and weights of the composite rule on [0, tau]."""
    edges = [0.0, tau * 2.0 ** -QUAD_LEVELS]
    edges += [tau * 2.0 ** -i for i in range(QUAD_LEVELS - 1, -1, -1)]
    nodes, weights = [], []
    for a, b in zip(edges[:-1], edges[1:]):
        h = (b - a) / QUAD_SPLIT
        for u in range(QUAD_SPLIT):
            lo = a + u * h
            nodes.append(lo + 0.5 * h * (GL_NODES + 1.0))
            weights.append(0.5 * h * GL_WEIGHTS)
    return np.concatenate(nodes), np.concatenate(weights)


def h_entry(H: np.ndarray, t: float) -> float:
    """(e^{t H})_{k,1}: last row, first column of the exponential."""
    return float(expm_pade13(H * t)[-1, 0])


def is_sym_tridiagonal(H: np.ndarray) -> bool:
    k = H.shape[0]
    return (np.array_equal(H, H.T) and
            not np.any(np.triu(H, 2)) and not np.any(np.tril(H, -2))) if k else True


def h_values(H: np.ndarray, ts: np.ndarray) -> np.ndarray:
    """(e^{t H})_{k,1} at every t of ts.  A symmetric tridiagonal H goes
    through its eigen-decomposition (LAPACK's tridiagonal solver), anything
    else through one Pade exponential per t."""
    k = H.shape[0]
    if k == 0:
        return np.zeros(len(ts))
    if is_sym_tridiagonal(H):
        theta, Q = sla.eigh_tridiagonal(np.diag(H).copy(), np.diag(H, -1).copy())
        wts = Q[-1, :] * Q[0, :]
        return np.array([float(np.sum(wts * np.exp(theta * t))) for t in ts])
    return np.array([h_entry(H, t) for t in ts])


def lemma1_integral(H: np.ndarray, tau: float, affine: bool = False) -> float:
    """int_0^tau w(t) |(e^{tH})_{k,1}| dt with w = 1, or w = tau - t for the
    augmented run."""
    x, w = quadrature_nodes(tau)
    vals = np.abs(h_values(H, x))
    if affine:
        vals = vals * (tau - x)
    return float(np.sum(w * vals))


def lemma1_bound(H, h_next, tau, lam_upper, affine=False) -> float:
    """The error bound of Lemma 1 for the normalised process (see the module
    docstring)."""
    if H.shape[0] == 0:
        return 0.0
    return float(h_next * math.exp(max(lam_upper, 0.0) * tau) * lemma1_integral(H, tau, affine))


def gershgorin_sym_upper(A) -> float:
    """An upper bound of lambda_max((A + A^T)/2): Gershgorin's bound of the
    symmetric part S with each |s_rc| = |a_rc + a_cr| / 2 taken as at most
    (|a_rc| + |a_cr|) / 2, i.e. max_r of a_rr plus half the absolute
    off-diagonal sums of row r and of column r.  For a symmetric A this is
    Gershgorin's bound of A itself."""
    import scipy.sparse as sp
    A = sp.csr_matrix(A)
    d = A.diagonal()
    absA = abs(A)
    row_off = np.asarray(absA.sum(axis=1)).ravel() - np.abs(d)
    col_off = np.asarray(absA.sum(axis=0)).ravel() - np.abs(d)
    return float(np.max(d + 0.5 * (row_off + col_off)))


def k_schedule(k0: int, kmax: int):
    """The checkpoints of Algorithms 2 and 4: k0, then k <- ceil(1.1 k) with
    1.1 k a double-precision product."""
    k = k0
    while k <= kmax:
        yield k
        k = math.ceil(1.1 * k)


def adaptive_lanczos(A, v, C, eps, tau, kmax, lam_upper, opnorm, affine=False):
    """Algorithm 4 with its error control: the Lanczos process of
    ``krylov.lanczos`` on v / |v| (beta0 = |v| is returned for the caller's
    scaling), and at every checkpoint k of ``k_schedule`` the Lemma 1 bound
    of T_k (diagonal alpha_1..alpha_k, off-diagonal beta_1..beta_{k-1}) with
    h_{k+1,k} = beta_k; the run stops at the first checkpoint whose bound is
    below eps.  When none is, it runs to kmax and keeps the last checkpoint's
    bound (inf when no checkpoint was reached).  A breakdown ends the run
    exactly (bound 0) at k_eff.  Returns dict(k_stop, bound, H = T at the
    stop, P = C V, beta0, k_eff, h = beta at the stop)."""
    v = np.asarray(v, np.float64)
    beta0 = math.sqrt(float(np.sum(v * v)))
    o = C.shape[0]
    if beta0 == 0.0 or kmax < 1:
        return {"k_stop": 0, "bound": 0.0, "H": np.zeros((0, 0)), "P": np.zeros((o, 0)), "beta0": 0.0,
                "k_eff": 0, "h": 0.0}
    checks = set(k_schedule(4, kmax))
    alpha, beta, cols = [], [], []
    q_old = np.zeros_like(v)
    q = v / beta0
    bound = math.inf

    def result(m, bnd):
        T = np.diag(alpha[:m]) + np.diag(beta[:m - 1], 1) + np.diag(beta[:m - 1], -1)
        return {"k_stop": m, "bound": bnd, "H": T, "P": np.stack(cols[:m], axis=1), "beta0": beta0,
                "k_eff": m, "h": float(beta[m - 1])}

    for m in range(1, kmax + 1):
        cols.append(np.asarray(C @ q).ravel())
        r = A @ q
        if beta:
            r = r - beta[-1] * q_old
        a = float(np.sum(q * r))
        r = r - a * q
        b = math.sqrt(float(np.sum(r * r)))
        alpha.append(a)
        beta.append(b)
        if b <= BREAKDOWN_FACTOR * EPS * opnorm:
            return result(m, 0.0)
        if m in checks:
            T = np.diag(alpha) + np.diag(beta[:-1], 1) + np.diag(beta[:-1], -1)
            bound = lemma1_bound(T, b, tau, lam_upper, affine)
            if bound < eps:
                return result(m, bound)
        q_old, q = q, r / b
    return result(kmax, bound)


def adaptive_arnoldi(A, v, C, eps, tau, kmax, lam_upper, opnorm, affine=False):
    """Algorithm 2 with its error control: the Arnoldi process of
    ``krylov.arnoldi`` on v / |v| to kmax, and at every checkpoint j of
    ``k_schedule`` (in order) the Lemma 1 bound of the leading block H_j with
    h_{j+1,j}; the first checkpoint below eps is the stop.  A breakdown at
    k_eff ends the run exactly (bound 0) unless an earlier checkpoint passed.
    Returns the dict of ``adaptive_lanczos``."""
    o = C.shape[0]
    res = arnoldi(A, v, kmax, C, opnorm=opnorm) if kmax >= 1 else None
    if res is None or res.k_eff == 0:
        return {"k_stop": 0, "bound": 0.0, "H": np.zeros((0, 0)), "P": np.zeros((o, 0)), "beta0": 0.0,
                "k_eff": 0, "h": 0.0}
    ke = res.k_eff
    broke = _breaks_down(res.h_next, opnorm)

    def h_after(j):
        return float(res.H[j, j - 1]) if j < ke else float(res.h_next)

    def result(j, bnd):
        return {"k_stop": j, "bound": bnd, "H": res.H[:j, :j].copy(), "P": res.P[:, :j].copy(),
                "beta0": res.beta0, "k_eff": j, "h": h_after(j)}

    bound = math.inf
    for j in k_schedule(4, kmax):
        if j > ke or (j == ke and broke):
            break
        bound = lemma1_bound(res.H[:j, :j], h_after(j), tau, lam_upper, affine)
        if bound < eps:
            return result(j, bound)
    if broke:
        return result(ke, 0.0)
    return result(ke, bound)


def adaptive_verify(problem, eps=1e-6, kmax=None, steps=None, dt=None, method="auto"):
    """Every run of a problem with the Krylov dimension chosen by the error
    control above (generator and center runs: Lanczos, or Arnoldi for a
    nonsymmetric A or method="arnoldi", on A; the augmented run: the same
    process from b, bordered by the augmented variable).  Returns
    dict(basis (S+1, o, nruns), roles, runs: dicts with k_stop, bound, dim
    (Krylov dimension used), k_eff, H (the Krylov matrix up to k_stop), h,
    beta0, affine, kmax (the run's cap), verdict) and lam (the Gershgorin
    bound used)."""
    from .krylov import box_check, build_runs, inf_norm, output_matrix, system_matrix
    if method == "auto":
        method = "lanczos" if problem.symmetric else "arnoldi"
    if method == "lanczos" and not problem.symmetric:
        raise ValueError("Lanczos needs a symmetric A")
    run_one = adaptive_lanczos if method == "lanczos" else adaptive_arnoldi
    steps = problem.steps if steps is None else steps
    dt = problem.dt if dt is None else dt
    kmax = problem.k if kmax is None else kmax
    A = system_matrix(problem)
    C = output_matrix(problem)
    opnorm = inf_norm(A)
    lam = gershgorin_sym_upper(A)
    tau = steps * dt
    runs = build_runs(problem)
    cols, info = [], []
    for run in runs:
        if run.role == "affine":
            r = run_one(A, problem.forcing(), C, eps, tau, kmax - 1, lam, opnorm, affine=True)
            m = r["H"].shape[0]
            Hb = np.zeros((m + 1, m + 1))
            Hb[1:, 1:] = r["H"]
            if m:
                Hb[1, 0] = r["beta0"]
            Pb = np.zeros((C.shape[0], m + 1))
            Pb[:, 1:] = r["P"]
            scale, dim = 1.0, m + 1
        else:
            r = run_one(A, run.start, C, eps, tau, kmax, lam, opnorm)
            Hb, Pb, scale, dim = r["H"], r["P"], r["beta0"], r["H"].shape[0]
        out = np.zeros((steps + 1, C.shape[0]))
        if dim > 0 and (run.role == "affine" or scale != 0.0):
            e1 = np.zeros(dim)
            e1[0] = 1.0
            for s in range(steps + 1):
                out[s] = scale * (Pb @ (expm_pade13(Hb * (s * dt)) @ e1))
        cols.append(out)
        info.append({"k_stop": r["k_stop"], "bound": r["bound"], "dim": dim, "k_eff": r["k_eff"], "H": r["H"],
                     "h": r["h"], "beta0": r["beta0"], "affine": run.role == "affine", "kmax": kmax - 1 if run.role == "affine"
                     else kmax})
    basis = np.stack(cols, axis=2)
    roles = [r.role for r in runs]
    zc = np.array([g.zc for g in problem.gens])
    rad = np.array([g.radius for g in problem.gens])
    return {"basis": basis, "roles": roles, "runs": info, "lam": lam,
            "verdict": box_check(basis, roles, zc, rad, problem.unsafe)}
