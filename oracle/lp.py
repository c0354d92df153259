"""Per-step safety LP (Section 2.1) in the initial-space coordinates.

TEST INFRASTRUCTURE ONLY (see the package docstring).

At time step s the reachable outputs are y = M_s z + f_s, with M_s the
generator columns of the basis C e^{A s dt} E and f_s the sum of its fixed
columns (center, forcing: coefficient 1).  The initial set is a polytope in
z: the generators' box |z_j - zc_j| <= r_j intersected with G z <= h (the
constraints I_x x0 <= iota_x of Section 2.1 written for x0 = E z).  The
unsafe set is a conjunction of halfspaces in the output space,
U y <= u (Section 3.1).  Step s is unsafe when

    { z : z in box, G z <= h, U (M_s z + f_s) <= u }

is non-empty (the LP of Section 2.1, whose x = e^{At} x0 equalities are
substituted through the basis); a feasible z is the counter-example of
Section 2.2.  The LP solver is SciPy's ``linprog`` (a library primitive).

Tolerance (the paper's LP solver works to 1e-6, Section 4.2): the decision
is made on the G and U rows a z <= b each divided by max(|a|_max, |b|), the
row's own magnitude; step s is unsafe when some z in the box violates no
scaled row by more than LP_TOL = 1e-6.  Scaling a row by a positive number
leaves the set unchanged, and it makes the tolerance independent of how U
and G are scaled; a solver's absolute tolerance on unscaled rows is not
(an output row whose basis entries are 1e-7 would be judged at the
solver's 1e-7 with a 100 % relative error).  A row whose coefficients
vanish against its right-hand side then reads 0 <= sign(b); a row of
magnitude below 1e-280 in both is 0 <= 0 and is dropped.  The decision
errs towards "unsafe" by at most LP_TOL.
"""
from __future__ import annotations

import numpy as np
from scipy.optimize import linprog


LP_TOL = 1e-6


def split_basis(basis_s: np.ndarray, roles):
    """(M_s, f_s) from one step's basis (o x ncols)."""
    gen = [i for i, r in enumerate(roles) if r == "gen"]
    fix = [i for i, r in enumerate(roles) if r != "gen"]
    return basis_s[:, gen], basis_s[:, fix].sum(axis=1)


def lp_feasible(M, f, zlo, zhi, G, h, U, u):
    """Exact-arithmetic feasibility of {z in [zlo, zhi], G z <= h,
    U (M z + f) <= u} as SciPy decides it (its own absolute tolerance).
    Returns (feasible, z) with z a feasible point (None when infeasible)."""
    d = M.shape[1]
    A = np.vstack([np.reshape(G, (len(h), d)), U @ M])
    b = np.concatenate([h, u - U @ f])
    if d == 0:
        ok = bool(np.all(b >= 0.0))
        return ok, (np.zeros(0) if ok else None)
    res = linprog(np.zeros(d), A_ub=A if A.size else None, b_ub=b if b.size else None,
                  bounds=list(zip(zlo, zhi)), method="highs")
    if res.status == 0:
        return True, np.asarray(res.x, np.float64)
    if res.status == 2:
        return False, None
    raise RuntimeError(f"linprog: {res.message}")


def lp_margin(M, f, zlo, zhi, G, h, U, u, with_point=False):
    """The smallest t with {z in box : a_i z - t <= b_i for every G and U
    row, each divided by max(|a_i|_max, |b_i|)}: negative when the set has
    an interior point, positive when it is empty.  With ``with_point`` also
    returns the minimising z."""
    d = M.shape[1]
    A = np.vstack([np.reshape(G, (len(h), d)), U @ M])
    b = np.concatenate([h, u - U @ f])
    amax = np.abs(A).max(axis=1) if (A.size and d) else np.zeros(A.shape[0])
    s = np.maximum(amax, np.abs(b))
    keep = s >= 1e-280
    A, b, s = A[keep], b[keep], s[keep]
    if A.shape[0] == 0:
        # no constraint: every box point qualifies; the centre of the box
        return (-np.inf, 0.5 * (np.asarray(zlo) + np.asarray(zhi))) if with_point else -np.inf
    A, b = A / s[:, None], b / s
    # variables (z, t): minimise t
    c = np.zeros(d + 1); c[d] = 1.0
    Aub = np.hstack([A, -np.ones((A.shape[0], 1))])
    res = linprog(c, A_ub=Aub, b_ub=b, bounds=list(zip(zlo, zhi)) + [(None, None)], method="highs")
    if res.status != 0:
        raise RuntimeError(f"linprog: {res.message}")
    t = float(res.x[d])
    return (t, np.asarray(res.x[:d], np.float64)) if with_point else t


def lp_check(basis: np.ndarray, roles, zc, radius, G, h, U, u):
    """The LP at every step s = 0..S, decided with LP_TOL on the scaled rows
    (see the module docstring).  Returns dict(first_step (-1 when safe), z
    (counter-example), y (its outputs M z + f), feasible (per-step bool),
    margin (per-step smallest scaled violation))."""
    zc = np.asarray(zc, np.float64); radius = np.asarray(radius, np.float64)
    zlo, zhi = zc - radius, zc + radius
    h = np.asarray(h, np.float64); u = np.asarray(u, np.float64)
    G = np.asarray(G, np.float64).reshape(h.size, zc.size)
    U = np.asarray(U, np.float64).reshape(u.size, basis.shape[1])
    feas = np.zeros(basis.shape[0], bool)
    margin = np.zeros(basis.shape[0])
    first, z_ce = -1, None
    for s in range(basis.shape[0]):
        M, f = split_basis(basis[s], roles)
        t, z = lp_margin(M, f, zlo, zhi, G, h, U, u, with_point=True)
        margin[s] = t
        feas[s] = t <= LP_TOL
        if feas[s] and first < 0:
            first, z_ce = s, z
    y = None
    if first >= 0:
        M, f = split_basis(basis[first], roles)
        y = M @ z_ce + f
    return {"first_step": first, "z": z_ce, "y": y, "feasible": feas, "margin": margin}
