"""The oracle's arithmetic.  See the package docstring: test infrastructure only.

Reductions (dot products and norms) are written as ``np.sum(a * b)``, which
NumPy evaluates by pairwise summation, so their rounding does not grow
linearly with n and does not depend on any thread count.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from fractions import Fraction
from typing import List, Optional

import numpy as np
import scipy.sparse as sp

# Breakdown rule (the paper only says the loop may stop when a norm is zero,
# Section 4.2): a step breaks down when the new vector's norm is at most
# BREAKDOWN_FACTOR * eps * ||Op||_inf, with ||Op||_inf the largest absolute
# row sum of the operator the run uses (A, or the augmented matrix for the
# affine run).  Rounding in Op @ v is of that size, so a smaller norm is zero
# up to rounding and the Krylov space is invariant.
BREAKDOWN_FACTOR = 1024.0
EPS = np.finfo(np.float64).eps


def _dot(a, b):
    return float(np.sum(a * b))


def _norm(a):
    return math.sqrt(float(np.sum(a * a)))


# ---------------------------------------------------------------------------
# Inputs -> operators
# ---------------------------------------------------------------------------

def system_matrix(problem) -> sp.csr_matrix:
    """A as a SciPy CSR matrix (a stencil problem is expanded to CSR)."""
    rowptr, colidx, vals = problem.csr()
    n = problem.n
    return sp.csr_matrix((np.asarray(vals, np.float64), np.asarray(colidx, np.int64),
                          np.asarray(rowptr, np.int64)), shape=(n, n))


def output_matrix(problem) -> sp.csr_matrix:
    """C (o x n) from the sparse output rows (Section 3.1)."""
    rows, cols, vals = [], [], []
    for r, seg in enumerate(problem.C):
        for lo, hi, w in zip(seg.lo, seg.hi, seg.w):
            idx = np.arange(lo, hi)
            rows.append(np.full(idx.size, r)); cols.append(idx); vals.append(np.full(idx.size, w))
    if rows:
        rows = np.concatenate(rows); cols = np.concatenate(cols); vals = np.concatenate(vals)
    return sp.csr_matrix((vals, (rows, cols)), shape=(problem.o, problem.n))


def augment(A: sp.spmatrix, b: np.ndarray) -> sp.csr_matrix:
    """Affine-to-linear transformation (Section 2.1): one more variable a with
    a' = 0 and a(0) = 1; the new matrix has b as its extra column and a zero
    extra row."""
    n = A.shape[0]
    bcol = sp.csr_matrix(np.asarray(b, np.float64).reshape(n, 1))
    top = sp.hstack([A, bcol])
    bottom = sp.csr_matrix((1, n + 1))
    return sp.vstack([top, bottom]).tocsr()


# ---------------------------------------------------------------------------
# Krylov processes (Section 4.2-4.3)
# ---------------------------------------------------------------------------

@dataclass
class RunResult:
    H: np.ndarray          # k_eff x k_eff Hessenberg (tridiagonal for Lanczos)
    P: np.ndarray          # o x k_eff projected basis C V_k
    beta0: float           # |v|
    h_next: float          # h_{k+1,k}
    k_eff: int             # Krylov dimension actually used (< k after breakdown)
    V: Optional[np.ndarray] = None   # n x k_eff basis, kept by Arnoldi only


def inf_norm(A) -> float:
    """Largest absolute row sum of a sparse or dense matrix."""
    if sp.issparse(A):
        return float(abs(A).sum(axis=1).max()) if A.shape[0] else 0.0
    return float(np.abs(A).sum(axis=1).max()) if A.shape[0] else 0.0


def _breaks_down(eta: float, opnorm: float) -> bool:
    return eta <= BREAKDOWN_FACTOR * EPS * opnorm


def arnoldi(A, v, k, C, reorth=True, keep_V=False, opnorm=None) -> RunResult:
    """Algorithm 1 (Arnoldi, modified Gram-Schmidt form) with a fixed number
    of iterations k.  The inner projection loop runs over the previous
    directions j = 1..i-1 (the printed bound j = 1..i would project the new
    vector on itself).  With ``reorth`` the projection loop is run a second
    time and its coefficients are added to H ("twice is enough").
    The start vector v is normalised here; beta0 = |v| multiplies the result
    (Eq. approx-formula)."""
    v = np.asarray(v, np.float64)
    beta0 = _norm(v)
    o = C.shape[0]
    if beta0 == 0.0:
        return RunResult(np.zeros((0, 0)), np.zeros((o, 0)), 0.0, 0.0, 0)
    opnorm = inf_norm(A) if opnorm is None else opnorm
    V = [v / beta0]
    H = np.zeros((k + 1, k))
    k_eff = k
    for i in range(1, k + 1):            # builds column i-1 of H, vector V[i]
        w = A @ V[i - 1]
        passes = 2 if reorth else 1
        for _ in range(passes):
            for j in range(i):
                hji = _dot(V[j], w)
                H[j, i - 1] += hji
                w = w - hji * V[j]
        eta = _norm(w)
        H[i, i - 1] = eta
        if _breaks_down(eta, opnorm):
            k_eff = i
            break
        V.append(w / eta)
    Vk = np.stack(V[:k_eff], axis=1)
    P = np.asarray(C @ Vk)
    return RunResult(H[:k_eff, :k_eff].copy(), P, beta0, float(H[k_eff, k_eff - 1]), k_eff,
                     Vk if keep_V else None)


def lanczos(A, v, k, C, opnorm=None) -> RunResult:
    """The symmetric Lanczos process of Section 4.3 (Algorithm 3) with the
    on-the-fly projection of Algorithm 4, fixed k (no error control).

    For symmetric A the Krylov basis obeys the three-term relation
        A q_j = beta_{j-1} q_{j-1} + alpha_j q_j + beta_j q_{j+1},
    with alpha_j = q_j^T A q_j and beta_j = |A q_j - alpha_j q_j - beta_{j-1} q_{j-1}|,
    so only two basis vectors are live at a time; each new q_j is projected
    on the output rows at once (P = C V, one column per step) and then
    dropped.  alpha and beta are collected in their own arrays and T_k, the
    symmetric tridiagonal matrix with diagonal alpha and off-diagonal beta,
    is formed at the end.  A step whose beta is zero up to rounding (the
    breakdown rule above) ends the process with an invariant Krylov space."""
    v = np.asarray(v, np.float64)
    beta0 = _norm(v)
    o = C.shape[0]
    if beta0 == 0.0:
        return RunResult(np.zeros((0, 0)), np.zeros((o, 0)), 0.0, 0.0, 0)
    opnorm = inf_norm(A) if opnorm is None else opnorm
    alpha, beta, cols = [], [], []
    q_old = np.zeros_like(v)
    q = v / beta0
    for _ in range(k):
        cols.append(np.asarray(C @ q).ravel())
        r = A @ q
        if beta:
            r = r - beta[-1] * q_old
        a = _dot(q, r)
        r = r - a * q
        b = _norm(r)
        alpha.append(a)
        beta.append(b)
        if _breaks_down(b, opnorm):
            break
        q_old, q = q, r / b
    m = len(alpha)
    T = np.diag(alpha) + np.diag(beta[:m - 1], 1) + np.diag(beta[:m - 1], -1)
    return RunResult(T, np.stack(cols, axis=1), beta0, float(beta[-1]), m)


# ---------------------------------------------------------------------------
# Small dense exponential: Pade [13/13] with scaling and squaring
# (N. J. Higham, "The scaling and squaring method for the matrix exponential
# revisited", SIAM J. Matrix Anal. Appl. 26(4), 2005)
# ---------------------------------------------------------------------------

THETA_13 = 5.371920351148152   # Higham 2005, largest 1-norm handled by degree 13 without scaling


def pade13_coefficients():
    """Coefficients of the [13/13] Pade numerator of e^x, scaled so the
    leading one is 1: c_j proportional to (2m-j)! m! / ((2m)! j! (m-j)!)."""
    m = 13
    c = [Fraction(math.factorial(2 * m - j) * math.factorial(m),
                  math.factorial(2 * m) * math.factorial(j) * math.factorial(m - j))
         for j in range(m + 1)]
    return [float(cj / c[m]) for cj in c]


_B13 = pade13_coefficients()


def expm_pade13(M: np.ndarray) -> np.ndarray:
    M = np.asarray(M, np.float64)
    k = M.shape[0]
    if k == 0:
        return np.zeros((0, 0))
    nrm = float(np.abs(M).sum(axis=0).max())
    s = 0
    if nrm > THETA_13:
        s = int(math.ceil(math.log2(nrm / THETA_13)))
    X = M / (2.0 ** s)
    I = np.eye(k)
    X2 = X @ X
    X4 = X2 @ X2
    X6 = X4 @ X2
    b = _B13
    U = X @ (X6 @ (b[13] * X6 + b[11] * X4 + b[9] * X2) + b[7] * X6 + b[5] * X4 + b[3] * X2 + b[1] * I)
    V = X6 @ (b[12] * X6 + b[10] * X4 + b[8] * X2) + b[6] * X6 + b[4] * X4 + b[2] * X2 + b[0] * I
    E = np.linalg.solve(V - U, V + U)
    for _ in range(s):
        E = E @ E
    return E


def project_steps(run: RunResult, dt: float, steps: int) -> np.ndarray:
    """y_s = beta0 * P * e^{H s dt} e_1 for s = 0..steps (Eq. approx-formula,
    projected as in Algorithm 4), one independent exponential per step.
    Returns (steps+1, o)."""
    o = run.P.shape[0]
    out = np.zeros((steps + 1, o))
    if run.k_eff == 0:
        return out
    e1 = np.zeros(run.k_eff); e1[0] = 1.0
    for s in range(steps + 1):
        w = expm_pade13(run.H * (s * dt)) @ e1
        out[s] = run.beta0 * (run.P @ w)
    return out


# ---------------------------------------------------------------------------
# Runs: one simulation per column of E (Section 4.1), after augmentation
# ---------------------------------------------------------------------------

@dataclass
class Run:
    role: str              # "gen" | "center" | "affine"
    start: np.ndarray      # start vector (length n, or n+1 for "affine")
    index: int             # generator number for role "gen"


def build_runs(problem) -> List[Run]:
    """Columns of E: each generator [g_j; 0], the fixed center [x_c; 0] when
    given, and the augmented variable's unit vector [0; 1] when b is given
    (Section 2.1 and 3.2).  The generator and center columns have a zero
    last entry, so their Krylov spaces under the augmented matrix are those
    of A itself; they are simulated with A (Lanczos for symmetric A).  The
    [0;1] column is simulated with the augmented matrix by Arnoldi."""
    n = problem.n
    runs = [Run("gen", g.seg.dense(n), j) for j, g in enumerate(problem.gens)]
    if problem.center is not None:
        runs.append(Run("center", np.asarray(problem.center, np.float64), -1))
    if problem.has_forcing:
        e = np.zeros(n + 1); e[n] = 1.0
        runs.append(Run("affine", e, -1))
    return runs


def krylov_run(problem, run: Run, A=None, Aaug=None, C=None, method="auto", k=None) -> RunResult:
    """One simulation.  Every run's breakdown test uses the scale ||A||_inf of
    the system matrix (the augmented run included), so all runs of a problem
    share one threshold."""
    A = system_matrix(problem) if A is None else A
    C = output_matrix(problem) if C is None else C
    k = problem.k if k is None else k
    opnorm = inf_norm(A)
    if run.role == "affine":
        Aaug = augment(A, problem.forcing()) if Aaug is None else Aaug
        Caug = sp.hstack([C, sp.csr_matrix((C.shape[0], 1))]).tocsr()
        return arnoldi(Aaug, run.start, k, Caug, opnorm=opnorm)
    if method == "arnoldi" or (method == "auto" and not problem.symmetric):
        return arnoldi(A, run.start, k, C, opnorm=opnorm)
    return lanczos(A, run.start, k, C, opnorm=opnorm)


# ---------------------------------------------------------------------------
# Per-step box check (Section 2.1 LP, for a box initial set)
# ---------------------------------------------------------------------------

def box_check(basis: np.ndarray, roles: List[str], zc: np.ndarray, radius: np.ndarray,
              unsafe: np.ndarray):
    """basis: (S+1, o, nruns) = C e^{A s dt} E.  Generator runs carry a box
    coefficient z_j in [zc_j - r_j, zc_j + r_j]; center and affine runs carry
    coefficient 1.  For each step and output row the reachable output range
    is an interval [mid - rad, mid + rad]; row r is violated when it meets
    the unsafe interval [lo_r, hi_r].  Returns a dict with the first
    violated (step, row) (-1 when safe), the counter-example z (the
    generator coefficients) and its output value, plus the per-step ranges.
    The counter-example is the point of the box whose output is nearest to
    the box center's output along the sign direction of the basis row."""
    S1, o, nr = basis.shape
    gen_idx = [i for i, r in enumerate(roles) if r == "gen"]
    fix_idx = [i for i, r in enumerate(roles) if r != "gen"]
    Mg = basis[:, :, gen_idx]                     # (S+1, o, ngen)
    mid = (Mg * zc[None, None, :]).sum(axis=2) + basis[:, :, fix_idx].sum(axis=2)
    rad = (np.abs(Mg) * radius[None, None, :]).sum(axis=2)
    lo_y, hi_y = mid - rad, mid + rad
    hit = (lo_y <= unsafe[None, :, 1]) & (hi_y >= unsafe[None, :, 0])
    result = {"first_step": -1, "row": -1, "y": float("nan"), "z": zc.copy(),
              "lo": lo_y, "hi": hi_y, "unsafe_mask": hit}
    if not hit.any():
        return result
    s, r = np.argwhere(hit)[0]                    # row-major: smallest step, then row
    m, rd = mid[s, r], rad[s, r]
    sgn = np.sign(Mg[s, r])
    lam, direction, y = 0.0, 0.0, m
    if m < unsafe[r, 0]:
        lam, direction = (unsafe[r, 0] - m) / rd, 1.0
    elif m > unsafe[r, 1]:
        lam, direction = (m - unsafe[r, 1]) / rd, -1.0
    z = zc + direction * lam * sgn * radius
    y = m + direction * lam * rd
    result.update(first_step=int(s), row=int(r), y=float(y), z=z)
    return result


def verify(problem, method="auto", k=None, steps=None, dt=None):
    """Whole path: runs -> Krylov -> per-step exponentials -> basis -> box
    check.  Returns dict(basis (S+1, o, nruns), roles, runs (RunResult),
    verdict)."""
    steps = problem.steps if steps is None else steps
    dt = problem.dt if dt is None else dt
    A = system_matrix(problem)
    C = output_matrix(problem)
    Aaug = augment(A, problem.forcing()) if problem.has_forcing else None
    runs = build_runs(problem)
    results = [krylov_run(problem, r, A=A, Aaug=Aaug, C=C, method=method, k=k) for r in runs]
    basis = np.stack([project_steps(res, dt, steps) for res in results], axis=2)
    roles = [r.role for r in runs]
    zc = np.array([g.zc for g in problem.gens])
    rad = np.array([g.radius for g in problem.gens])
    verdict = box_check(basis, roles, zc, rad, problem.unsafe)
    return {"basis": basis, "roles": roles, "runs": results, "verdict": verdict}
