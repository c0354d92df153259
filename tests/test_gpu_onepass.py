"""The one-pass Lanczos step (FP64 three-vector Lanczos, one launch per
iteration over the pair buffers (u_{j-1}, r_j)) against the FP64 oracle and
against the two-launch step it replaces (KRY_ONEPASS=0): on the sliced-ELL
CSR mat-vec (used there on request, KRY_ONEPASS=1), the row stencil and the
marching stencil (forced on small grids with KRY_STENCIL_MARCH=1), with
batches of 1 to 8 runs; and the hand-back to the two-launch step when a
run's norm expansion cancels (an invariant Krylov space)."""
import math
import os
from contextlib import contextmanager

import numpy as np
import pytest
import torch  # noqa: F401

import oracle
import workloads as W
from paper_1804_01583_amd import kry
from tests.gpu_helpers import assert_basis_parity, assert_krylov_parity, gpu_verify, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _general_path(monkeypatch):
    # these kernels belong to the general path: small systems would take the
    # persistent small-system kernel instead
    monkeypatch.setenv("KRY_SMALL", "0")


@contextmanager
def env(**kv):
    old = {k: os.environ.get(k) for k in kv}
    os.environ.update({k: str(v) for k, v in kv.items()})
    try:
        yield
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def _profiled(problem, **kw):
    kry.profile_enable(True)
    kry.profile_reset()
    try:
        got = gpu_verify(problem, **kw)
        counts = {n: kry.profile_read(n)[0] for n in kry.profile_names()}
    finally:
        kry.profile_enable(False)
    return got, counts


def _check(problem, step_kernel, **kw):
    # KRY_ONEPASS=1: the step on CSR systems too (by default stencils only)
    require_gpu()
    ref = oracle.verify(problem)
    with env(KRY_ONEPASS=1):
        got, counts = _profiled(problem, **kw)
    assert counts[step_kernel] > 0, counts
    assert counts["sweep"] == 0, "a batch was handed back to the two-launch step"
    for g, r in zip(got["runs"], ref["runs"]):
        assert_krylov_parity(g, r)
    worst = assert_basis_parity(got["basis"], ref["basis"])
    assert got["verdict"]["first_step"] == ref["verdict"]["first_step"]
    with env(KRY_ONEPASS=0):
        two, counts2 = _profiled(problem, **kw)
    assert counts2[step_kernel] == 0 and counts2["sweep"] > 0
    # the same vectors up to the rounding of |u_j| (expanded vs summed)
    scale = np.abs(two["basis"]).max(axis=0)
    diff = np.abs(got["basis"] - two["basis"]).max(axis=0)
    assert np.all(diff <= 1e-12 * np.where(scale > 0, scale, 1.0)), (diff, scale)
    print(f"  worst relative error vs oracle {worst:.2e}", flush=True)
    return got, ref


def test_onepass_sliced_ell_with_center_and_forcing():
    p = W.small_heat3d(m=14, k=24, steps=120)
    c = np.zeros(p.n)
    c[100:300] = 0.3
    p.center = c
    _check(p, "lz1_sell")


@pytest.mark.parametrize("ngen,forcing,o", [(1, False, 3), (3, True, 2), (7, True, 2)])
def test_onepass_batches_of_one_to_eight(ngen, forcing, o):
    # one run alone; 3 + forcing = 4 runs; 7 + forcing = 8 runs in one launch
    m = 15
    p = W.small_heat3d(m=m, k=20, steps=60)
    gens = []
    for g in range(ngen):
        x0 = (2 * g) % (m - 3)
        gens.append(W.Generator(W.box_segments((m, m, m), ((x0, x0 + 2), (g % 5, g % 5 + 4), (1, 6)), 1.0),
                                zc=1.0 + 0.1 * g, radius=0.05))
    p.gens = gens
    p.C = p.C[:o]
    p.unsafe = p.unsafe[:o]
    if not forcing:
        p.b = None
    got, _ = _check(p, "lz1_sell")
    assert len(got["roles"]) == ngen + (1 if forcing else 0)


def test_onepass_row_stencil():
    p = W.small_heat3d(m=13, k=22, steps=80)
    ps = W.Problem("stencil", p.n, "stencil7", True, p.gens, p.C, p.unsafe, k=p.k, dt=p.dt, steps=p.steps,
                   b=p.b, grid=(13, 13, 13), coef=p.meta["coef"])
    _check(ps, "lz1_stencil")


@pytest.mark.parametrize("grid", [(37, 11, 19), (8, 30, 30), (9, 35, 130)])
def test_onepass_marching_stencil_forced(grid):
    # the marching kernel on a small grid (forced): nx not a multiple of its
    # three-plane unroll, dead lanes in the last column block, dead waves in
    # the last row tile (16 rows), several tiles both ways (35 rows, 130
    # columns against 60 per tile), outputs whose segments start mid-block
    # for the projection kernel
    nx, ny, nz = grid
    n = nx * ny * nz
    h = 1.0 / (max(grid) + 1)
    c = 0.01 / h**2
    gen = W.box_segments(grid, ((0, 4), (2, 7), (3, 9)), 1.0)
    fb = W.box_segments(grid, ((nx - 5, nx - 1), (ny - 6, ny - 2), (1, 5)), 0.1)
    C = [W.box_segments(grid, ((1, 6), (2, 8), (2, 12)), 1.0 / 300), W.box_segments(grid, ((nx - 7, nx), (0, ny), (0, 6)), 0.01)]
    p = W.Problem("march", n, "stencil7", True, [W.Generator(gen, zc=1.0, radius=0.1)], C,
                  np.array([[0.4, math.inf], [math.inf, math.inf]]), k=18, dt=0.01, steps=70,
                  b_seg=fb, grid=grid, coef=(-6 * c, c, c, c))
    with env(KRY_STENCIL_MARCH=1):
        _check(p, "lz1_march")


def test_onepass_hands_back_on_an_invariant_space():
    # a sine mode is an eigenvector: after one step the new direction is
    # rounding noise, which the expanded norm cannot resolve; the batch is
    # computed again two-pass and breaks down exactly
    require_gpu()
    p = W.heat1d(steps=50)
    n = p.n
    h = 1.0 / (n + 1)
    p.gens = [W.Generator(W.segments_from_ranges([(0, 10)], 1.0), 0.0, 1.0)]
    p.center = np.sin(3 * math.pi * np.arange(1, n + 1) * h)
    p.C = [W.segments_from_ranges([(90, 111)], 1.0 / 21.0)]
    ref = oracle.verify(p)
    with env(KRY_ONEPASS=1):
        got, counts = _profiled(p)
    assert counts["lz1_sell"] > 0 and counts["sweep"] > 0
    assert [r["k_eff"] for r in got["runs"]] == [r.k_eff for r in ref["runs"]]
    assert got["runs"][1]["k_eff"] == 1
    assert_basis_parity(got["basis"], ref["basis"])


def test_onepass_plain_lanczos_large_k():
    # the three-vector process of Algorithm 4 at k = 150 (dense small stage)
    require_gpu()
    p = W.heat3d_paper(m=14)
    p.k = 150
    p.steps = 200
    with env(KRY_ONEPASS=1):
        got, counts = _profiled(p, method=kry.KRY_LANCZOS_PLAIN)
    assert counts["lz1_sell"] == 150 and counts["sweep"] == 0
    with env(KRY_ONEPASS=0):
        two = gpu_verify(p, method=kry.KRY_LANCZOS_PLAIN)
    scale = np.abs(two["basis"]).max(axis=0)
    diff = np.abs(got["basis"] - two["basis"]).max(axis=0)
    assert np.all(diff <= 1e-10 * np.where(scale > 0, scale, 1.0)), (diff, scale)
