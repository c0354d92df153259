"""Full-size parity for the matrix-free 3D heat system (1000^3 = 10^9 states,
Lanczos k = 20, 500 steps, FP64) through the C ABI.

The oracle cannot run 10^9 states, but the computed quantity is local: after j
Krylov steps from a start vector supported in a box, every basis vector is
supported within grid distance j of that box (A is a 7-point stencil).  So
each run equals the same run on the sub-grid spanned by its start box dilated
by k + 1 cells, with outputs restricted to that sub-grid and exact zeros
outside it.  The oracle solves those sub-grid problems (a few million states)
and the full-size GPU result must match them within the parity bound."""
import math

import numpy as np
import pytest
import torch  # noqa: F401

import oracle
import workloads as W
from tests.gpu_helpers import assert_basis_parity, gpu_verify, require_gpu

pytestmark = pytest.mark.gpu


def _clip_box(box, lo, hi):
    return tuple((max(a, l), min(b, h)) for (a, b), l, h in zip(box, lo, hi))


def _sub_problem(full, start_box, role, k):
    m = full.meta["m"]
    lo = [max(a - (k + 1), 0) for a, _ in start_box]
    hi = [min(b + (k + 1), m) for _, b in start_box]
    grid = tuple(h - l for l, h in zip(lo, hi))
    shift = lambda box: tuple((a - l, b - l) for (a, b), l in zip(box, lo))   # noqa: E731
    C = []
    mid = m // 2
    gcount = int(np.prod([b - a for a, b in full.meta["gen_box"]]))
    for q, box in enumerate([((mid, mid + 1),) * 3, full.meta["gen_box"]]):
        cb = _clip_box(box, lo, hi)
        if all(b > a for a, b in cb):
            w = 1.0 if q == 0 else 1.0 / gcount
            C.append(W.box_segments(grid, shift(cb), w))
        else:
            C.append(None)
    live = [c for c in C if c is not None]
    if not live:
        return None, C
    sb = shift(start_box)
    gens, bseg = [], None
    if role == "gen":
        gens = [W.Generator(W.box_segments(grid, sb, 1.0), zc=1.0, radius=0.1)]
    else:
        bseg = W.box_segments(grid, sb, 0.1)
    p = W.Problem("sub", int(np.prod(grid)), "stencil7", True, gens, live,
                  np.array([[math.inf, math.inf]] * len(live)), k=full.k, dt=full.dt, steps=full.steps,
                  b_seg=bseg, grid=grid, coef=full.coef)
    return p, C


@pytest.mark.parametrize("m", [200, 1000])
def test_heat3d_stencil_full_size_by_locality(m):
    require_gpu()
    full = W.heat3d_stencil(m=m)
    print(f"[gpu] heat3d_stencil m={m} n={full.n} k={full.k} steps={full.steps}", flush=True)
    got = gpu_verify(full, workspace="library")
    assert got["roles"] == ["gen", "affine"]
    for r, (role, box) in enumerate([("gen", full.meta["gen_box"]), ("affine", full.meta["forcing_box"])]):
        sub, C = _sub_problem(full, box, role, full.k)
        if sub is None:
            assert np.all(got["basis"][:, :, r] == 0.0)
            continue
        ref = oracle.verify(sub)
        col = 0
        for q, c in enumerate(C):
            if c is None:
                assert np.all(got["basis"][:, q, r] == 0.0), f"row {q} run {r} should be structurally zero"
            else:
                assert_basis_parity(got["basis"][:, q:q + 1, r:r + 1], ref["basis"][:, col:col + 1, 0:1])
                col += 1
        assert got["runs"][r]["k_eff"] == ref["runs"][0].k_eff
