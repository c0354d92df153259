"""Block Krylov simulation of several generators at once: test infrastructure
only (see the package docstring).

The paper simulates one column of E at a time (Section 4.1).  Running p
columns together as one block Krylov space

    K_k(A, G) = span{G, A G, ..., A^{k-1} G},      G = [g_1 .. g_p]  (n x p)

turns every mat-vec into a product with p vectors and every orthogonalisation
into a dense p-wide contraction.  The approximant is the Galerkin one of
Section 4.2 written for a block start: with G = V_1 R_0 (thin QR) and an
orthonormal basis V = [V_1 .. V_k] of the block space, H = V^T A V,

    C e^{A t} G  ~  C V e^{H t} E_1 R_0,      E_1 = first p columns of I_{pk}.

It is exact when the block space is A-invariant (for instance when pk >= n).

Block Arnoldi here is Algorithm 1 with blocks in place of vectors: block
modified Gram-Schmidt against V_1..V_i, run twice with the second pass's
coefficients added to H (as in ``krylov.arnoldi``), and each new block
orthonormalised by a Householder QR whose R has a non-negative diagonal, so
V and H are unique.  A block whose R has a diagonal entry at most
1024 eps ||A||_inf ends the run (the block space has become invariant in at
least one direction; the run keeps the blocks before it)."""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import numpy as np

from .krylov import BREAKDOWN_FACTOR, EPS, box_check, expm_pade13, inf_norm, output_matrix, system_matrix


@dataclass
class BlockResult:
    H: np.ndarray          # (p k_eff) x (p k_eff) block upper Hessenberg
    P: np.ndarray          # o x (p k_eff): C V
    R0: np.ndarray         # p x p upper triangular, G = V_1 R0
    h_next: np.ndarray     # p x p block H_{k+1,k}
    k_eff: int             # number of blocks used
    p: int
    V: Optional[np.ndarray] = None   # n x (p k_eff) basis (keep_V)


def qr_posdiag(W: np.ndarray):
    """Thin Householder QR (LAPACK through numpy) with the signs fixed so
    that diag(R) >= 0."""
    Q, R = np.linalg.qr(W, mode="reduced")
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    return Q * s[None, :], R * s[:, None]


def block_arnoldi(A, G: np.ndarray, k: int, C, keep_V=False, opnorm=None) -> BlockResult:
    """k block steps from the start block G (n x p)."""
    G = np.asarray(G, np.float64)
    n, p = G.shape
    opnorm = inf_norm(A) if opnorm is None else opnorm
    tau = BREAKDOWN_FACTOR * EPS * opnorm
    V1, R0 = qr_posdiag(G)
    d0 = np.abs(np.diag(R0))
    if p == 0 or d0.min() <= BREAKDOWN_FACTOR * EPS * d0.max():
        # a zero or dependent start column: the block method needs a full-rank start
        raise ValueError("block start is rank deficient")
    V = [V1]
    H = np.zeros((p * (k + 1), p * k))
    k_eff = k
    for i in range(k):                   # block column i, new block V[i+1]
        W = np.asarray(A @ V[i])
        for _ in range(2):
            for j in range(i + 1):
                Hji = V[j].T @ W
                H[j * p:(j + 1) * p, i * p:(i + 1) * p] += Hji
                W = W - V[j] @ Hji
        Q, R = qr_posdiag(W)
        H[(i + 1) * p:(i + 2) * p, i * p:(i + 1) * p] = R
        if np.abs(np.diag(R)).min() <= tau:
            k_eff = i + 1
            break
        V.append(Q)
    m = p * k_eff
    Vk = np.concatenate(V[:k_eff], axis=1)
    P = np.asarray(C @ Vk)
    h_next = H[m:m + p, m - p:m].copy()
    return BlockResult(H[:m, :m].copy(), P, R0, h_next, k_eff, p, Vk if keep_V else None)


def block_project_steps(res: BlockResult, dt: float, steps: int) -> np.ndarray:
    """y_s = C V e^{H s dt} E_1 R_0 for s = 0..steps, one independent
    exponential per step.  Returns (steps+1, o, p)."""
    o = res.P.shape[0]
    p = res.p
    out = np.zeros((steps + 1, o, p))
    for s in range(steps + 1):
        E = expm_pade13(res.H * (s * dt))
        out[s] = res.P @ (E[:, :p] @ res.R0)
    return out


def block_verify(problem, p=16, k=None, steps=None, dt=None):
    """Generators in blocks of p (the last block may be narrower), each block
    one block Krylov run.  Returns dict(basis (S+1, o, ngen), roles, blocks)
    with the generator columns in order."""
    if problem.center is not None or problem.has_forcing:
        raise ValueError("block runs cover generator columns only")
    steps = problem.steps if steps is None else steps
    dt = problem.dt if dt is None else dt
    k = problem.k if k is None else k
    A = system_matrix(problem)
    C = output_matrix(problem)
    opnorm = inf_norm(A)
    n = problem.n
    cols, blocks = [], []
    for b0 in range(0, len(problem.gens), p):
        gens = problem.gens[b0:b0 + p]
        G = np.stack([g.seg.dense(n) for g in gens], axis=1)
        res = block_arnoldi(A, G, k, C, opnorm=opnorm)
        blocks.append(res)
        cols.append(block_project_steps(res, dt, steps))
    basis = np.concatenate(cols, axis=2)
    roles = ["gen"] * basis.shape[2]
    zc = np.array([g.zc for g in problem.gens])
    rad = np.array([g.radius for g in problem.gens])
    verdict = box_check(basis, roles, zc, rad, problem.unsafe)
    return {"basis": basis, "roles": roles, "blocks": blocks, "verdict": verdict}
