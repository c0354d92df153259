"""Basis matrix by simulation of the transposed dynamics (Section 4.1).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The basis matrix is C e^{At} E = (E^T e^{A^T t} C^T)^T, so instead of one
simulation per column of E there is one per row of C: x' = A^T x from the
output row c_q, projected on the rows of E^T.  The projection is the one of
Algorithm 4 with E^T in place of C (Section 4.3 says so for the transposed
case).

Affine systems (Section 2.1).  The columns of E live in the augmented space
(x, a): the generators and the center are [g; 0] and [x_c; 0], the forcing
adds [0; 1].  The transposed augmented matrix is [[A^T, 0], [b^T, 0]]; from
[c_q; 0] the first n entries follow A^T alone and the last one integrates b^T
of them over time.  The paper does not spell out the Krylov form of this run;
the reading taken here is the Galerkin projection of the transposed augmented
system on span{[v_1; 0], ..., [v_k; 0], [0; 1]}, with v_1..v_k the Krylov
basis of A^T from c_q.  The projected matrix is [[H, 0], [b^T V, 0]] (size
k + 1) and the projected start is [|c_q| e_1; 0], so the forcing costs one
projection row (b) and one exponential of size k + 1 per output row.
"""
from __future__ import annotations

from typing import List

import numpy as np
import scipy.sparse as sp

from .krylov import arnoldi, box_check, expm_pade13, inf_norm, lanczos, system_matrix


def initial_rows(problem) -> (sp.csr_matrix, List[str]):
    """Rows of E^T restricted to the first n coordinates, in the column order
    the basis uses everywhere: one per generator, the center when given, and
    b when the system is affine (the [0; 1] column of E enters through the
    b^T border of the transposed augmented matrix, so its row here is b, the
    row that border needs).  Returns (rows, roles)."""
    n = problem.n
    rows, roles = [], []
    for g in problem.gens:
        rows.append(g.seg.dense(n)); roles.append("gen")
    if problem.center is not None:
        rows.append(np.asarray(problem.center, np.float64)); roles.append("center")
    if problem.has_forcing:
        rows.append(problem.forcing()); roles.append("affine")
    R = sp.csr_matrix(np.stack(rows)) if rows else sp.csr_matrix((0, n))
    return R, roles


def transposed_runs(problem, method="auto", k=None):
    """One Krylov simulation of A^T per output row c_q (Section 4.1), each
    projected on the rows of ``initial_rows`` as it goes (Algorithm 4 with
    E^T for C).  Lanczos when A is symmetric (A^T = A), else Arnoldi.  The
    breakdown scale is ||A^T||_inf, that of the operator the runs use."""
    k = problem.k if k is None else k
    At = system_matrix(problem).T.tocsr()
    R, roles = initial_rows(problem)
    opnorm = inf_norm(At)
    out = []
    for seg in problem.C:
        c = seg.dense(problem.n)
        if method == "arnoldi" or (method == "auto" and not problem.symmetric):
            out.append(arnoldi(At, c, k, R, opnorm=opnorm))
        else:
            out.append(lanczos(At, c, k, R, opnorm=opnorm))
    return out, roles


def transposed_steps(run, roles, dt, steps) -> np.ndarray:
    """Values of E^T e^{A^T s dt} c_q for s = 0..steps, one independent
    exponential per step (Eq. approx-formula).  Without forcing this is
    beta0 P e^{H s dt} e_1.  With forcing the projected transposed augmented
    matrix M = [[H, 0], [p_b^T, 0]] (p_b the b row of P = E^T V) is
    exponentiated from [beta0 e_1; 0]: its first k entries give the
    generator and center values through P, its last entry is the forcing
    column's value.  Returns (steps + 1, len(roles))."""
    ncol = len(roles)
    out = np.zeros((steps + 1, ncol))
    m = run.k_eff
    if m == 0:
        return out
    affine = "affine" in roles
    fixed = [i for i, r in enumerate(roles) if r != "affine"]
    Pf = run.P[fixed, :]
    if affine:
        M = np.zeros((m + 1, m + 1))
        M[:m, :m] = run.H
        M[m, :m] = run.P[roles.index("affine"), :]
        x0 = np.zeros(m + 1); x0[0] = run.beta0
        for s in range(steps + 1):
            w = expm_pade13(M * (s * dt)) @ x0
            out[s, fixed] = Pf @ w[:m]
            out[s, roles.index("affine")] = w[m]
    else:
        e1 = np.zeros(m); e1[0] = 1.0
        for s in range(steps + 1):
            out[s, fixed] = run.beta0 * (Pf @ (expm_pade13(run.H * (s * dt)) @ e1))
    return out


def verify_transposed(problem, method="auto", k=None, steps=None, dt=None):
    """The whole path by the transposed route: o simulations instead of one
    per column of E, the basis C e^{A s dt} E recovered by transposition,
    then the same per-step box check as the forward route.  Returns the
    same dict as ``verify``: basis (S+1, o, ncols), roles, runs, verdict."""
    steps = problem.steps if steps is None else steps
    dt = problem.dt if dt is None else dt
    runs, roles = transposed_runs(problem, method=method, k=k)
    # row q of the basis at step s is the transposed run q's projected state
    basis = np.stack([transposed_steps(r, roles, dt, steps) for r in runs], axis=1)
    zc = np.array([g.zc for g in problem.gens])
    rad = np.array([g.radius for g in problem.gens])
    verdict = box_check(basis, roles, zc, rad, problem.unsafe)
    return {"basis": basis, "roles": roles, "runs": runs, "verdict": verdict}
