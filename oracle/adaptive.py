"""A-posteriori error control of the Krylov dimension (paper Section 4.2,
Lemma 1 and the red lines of Algorithms 2 and 4): test infrastructure only
(see the package docstring).

Lemma 1 (for e^{-tau B} v, |v| = 1, Arnoldi of B): the error is at most
h_{k+1,k} e^{-min(nu(B), 0) tau} * integral_0^tau |e_k^T e^{-t H^B_k} e_1| dt,
nu(B) the smallest eigenvalue of (B + B^T)/2.  The paper feeds B = -A to get
e^{tau A} v.  Arnoldi of -A has the same vectors as Arnoldi of A up to signs,
so |e_k^T e^{-t H^B_k} e_1| = |(e^{t H_k})_{k,1}| with H_k from A itself, and
-nu(-A) = lambda_max((A + A^T)/2).  With |v| = beta0:

    bound(tau) = beta0 h_{k+1,k} e^{max(lambda, 0) tau} int_0^tau |(e^{t H_k})_{k,1}| dt,

lambda any upper bound of lambda_max((A + A^T)/2) (Gershgorin here).

The augmented run approximates x(t) = int_0^t e^{As} b ds by integrating the
Lanczos approximation of e^{As} b (the bordered Krylov matrix does exactly
that), so its error is at most int_0^tau bound_b(s) ds
    = |b| h e^{max(lambda,0) tau} int_0^tau (tau - t) |(e^{t T})_{k,1}| dt
with T and h from the Lanczos process started at b.

The integral is evaluated by one fixed rule, the definition both sides
implement: composite 8-point Gauss-Legendre on [0, tau 2^-L] and on each
[tau 2^-(i+1), tau 2^-i], i = 0..L-1, every interval split into U equal
parts (L = 40, U = 8).  The geometric intervals resolve the fast transient
of h near t = 0 that a uniform grid misses.

The Krylov dimension is chosen as in Algorithms 2 and 4: check at k = 4,
then k <- ceil(1.1 k), stop at the first k whose bound is below the target.
"""
from __future__ import annotations

import math

import numpy as np

from .krylov import BREAKDOWN_FACTOR, EPS, expm_pade13

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


def lemma1_integral(H: np.ndarray, tau: float, affine: bool = False) -> float:
    """int_0^tau w(t) |(e^{tH})_{k,1}| dt with w = 1, or w = tau - t for the
    augmented run."""
    x, w = quadrature_nodes(tau)
    vals = np.array([abs(h_entry(H, t)) for t in x])
    if affine:
        vals = vals * (tau - x)
    return float(np.sum(w * vals))


def lemma1_bound(H, h_next, beta0, tau, lam_upper, affine=False) -> float:
    """The error bound of Lemma 1 (see the module docstring)."""
    if H.shape[0] == 0:
        return 0.0
    return float(beta0 * h_next * math.exp(max(lam_upper, 0.0) * tau) * lemma1_integral(H, tau, affine))


def gershgorin_sym_upper(A) -> float:
    """An upper bound of lambda_max((A + A^T)/2): max_i of the diagonal plus
    the absolute off-diagonal row sum of the symmetric part."""
    import scipy.sparse as sp
    S = 0.5 * (sp.csr_matrix(A) + sp.csr_matrix(A).T)
    d = S.diagonal()
    off = np.asarray(abs(S).sum(axis=1)).ravel() - np.abs(d)
    return float(np.max(d + off))


def k_schedule(k0: int, kmax: int):
    """The checkpoints of Algorithms 2 and 4: k0, then k <- ceil(1.1 k)."""
    k = k0
    while k <= kmax:
        yield k
        k = (11 * k + 9) // 10          # ceil(1.1 k) in exact integer arithmetic


def adaptive_lanczos(A, v, C, eps, tau, kmax, lam_upper, opnorm, affine=False):
    """Algorithm 4 with error control: Lanczos from v (|v| = beta0); at each
    checkpoint k the bound uses T_k and h = beta_k.  Returns dict(k_stop,
    bound, H, P, beta0, k_eff, h = h_{k+1,k} at the stop).  k_stop = kmax (bound above eps) when no
    checkpoint reaches the target; a breakdown ends the run exactly
    (bound 0) at k_eff."""
    v = np.asarray(v, np.float64)
    beta0 = math.sqrt(float(np.sum(v * v)))
    o = C.shape[0]
    if beta0 == 0.0:
        return {"k_stop": 0, "bound": 0.0, "H": np.zeros((0, 0)), "P": np.zeros((o, 0)), "beta0": 0.0,
                "k_eff": 0, "h": 0.0}
    checks = set(k_schedule(4, kmax))
    H = np.zeros((kmax + 1, kmax))
    P = np.zeros((o, kmax + 1))
    v_prev, v_cur = None, v / beta0
    P[:, 0] = C @ v_cur
    bound = math.inf
    for i in range(1, kmax + 1):
        w = A @ v_cur
        if i > 1:
            H[i - 2, i - 1] = H[i - 1, i - 2]
            w = w - H[i - 2, i - 1] * v_prev
        H[i - 1, i - 1] = float(np.sum(v_cur * w))
        w = w - H[i - 1, i - 1] * v_cur
        eta = math.sqrt(float(np.sum(w * w)))
        H[i, i - 1] = eta
        if eta <= BREAKDOWN_FACTOR * EPS * opnorm:
            return {"k_stop": i, "bound": 0.0, "H": H[:i, :i].copy(), "P": P[:, :i].copy(), "beta0": beta0,
                    "k_eff": i, "h": eta}
        if i in checks:
            bound = lemma1_bound(H[:i, :i], eta, beta0, tau, lam_upper, affine)
            if bound < eps:
                return {"k_stop": i, "bound": bound, "H": H[:i, :i].copy(), "P": P[:, :i].copy(), "beta0": beta0,
                        "k_eff": i, "h": eta}
        v_prev, v_cur = v_cur, w / eta
        P[:, i] = C @ v_cur
    return {"k_stop": kmax, "bound": bound, "H": H[:kmax, :kmax].copy(), "P": P[:, :kmax].copy(), "beta0": beta0,
            "k_eff": kmax, "h": float(H[kmax, kmax - 1])}


def adaptive_verify(problem, eps=1e-6, kmax=None, steps=None, dt=None):
    """Every run of a symmetric problem with the Krylov dimension chosen by
    the error control above (generator and center runs: Lanczos on A; the
    augmented run: Lanczos on A from b, bordered by the augmented variable).
    Returns dict(basis (S+1, o, nruns), roles, runs: dicts with k_stop,
    bound, dim (Krylov dimension used), k_eff, H (the Lanczos matrix up to
    k_stop), h, beta0, affine, kmax (the run's cap), verdict) and lam (the
    Gershgorin bound used)."""
    from .krylov import box_check, build_runs, inf_norm, output_matrix, system_matrix
    if not problem.symmetric:
        raise ValueError("the error-controlled path here is Lanczos (symmetric A)")
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
            r = adaptive_lanczos(A, problem.forcing(), C, eps, tau, kmax - 1, lam, opnorm, affine=True)
            m = r["H"].shape[0]
            Hb = np.zeros((m + 1, m + 1))
            Hb[1:, 1:] = r["H"]
            if m:
                Hb[1, 0] = r["beta0"]
            Pb = np.zeros((C.shape[0], m + 1))
            Pb[:, 1:] = r["P"]
            scale, dim = 1.0, m + 1
        else:
            r = adaptive_lanczos(A, run.start, C, eps, tau, kmax, lam, opnorm)
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
