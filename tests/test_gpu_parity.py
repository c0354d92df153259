"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the
same seeded inputs.  Bound: relative 1e-10 per (output row, run), rows that
the oracle gives as exactly zero must be exactly zero, identical verdicts."""
import math

import numpy as np
import pytest
import torch  # noqa: F401  (imported at collection so the first test does not pay for it)

import oracle
import workloads as W
from tests.gpu_helpers import (RTOL, assert_basis_parity, assert_krylov_parity, assert_verdict_parity,
                               gpu_verify, require_gpu)

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True, params=["small", "general"])
def _path(request, monkeypatch):
    # every test on both FP64 Lanczos paths: the persistent small-system
    # kernel (the default up to 2048 rows) and the general launches
    if request.param == "general":
        monkeypatch.setenv("KRY_SMALL", "0")
    else:
        monkeypatch.delenv("KRY_SMALL", raising=False)


def _compare(problem, method="auto", **kw):
    require_gpu()
    ref = oracle.verify(problem, method=method, k=kw.get("k"), steps=kw.get("steps"), dt=kw.get("dt"))
    got = gpu_verify(problem, **kw)
    assert got["roles"] == ref["roles"]
    for g, r in zip(got["runs"], ref["runs"]):
        assert_krylov_parity(g, r)
    worst = assert_basis_parity(got["basis"], ref["basis"])
    assert_verdict_parity(got["verdict"], ref["verdict"], ref["basis"])
    print(f"  worst relative error {worst:.2e}", flush=True)
    return got, ref


def test_heat1d_config_literal():
    # 1D heat n=200, k=30, 10 generators, 1000 steps: outputs structurally zero
    got, ref = _compare(W.heat1d())
    assert np.all(ref["basis"] == 0.0) and np.all(got["basis"] == 0.0)
    assert got["verdict"]["first_step"] == -1


def test_heat1d_reachable_output():
    # the same system with an output region the Krylov space reaches
    p = W.heat1d(steps=300)
    p.C = [W.segments_from_ranges([(3, 14)], 1.0 / 11.0), W.segments_from_ranges([(0, 1), (30, 34)], 0.5)]
    p.unsafe = np.array([[0.3, math.inf], [-math.inf, -5.0]])
    got, ref = _compare(p, dt=2e-4)
    assert np.abs(ref["basis"]).max() > 0.01


@pytest.mark.parametrize("m,k", [(12, 20), (17, 33)])
def test_small_heat3d_with_forcing(m, k):
    p = W.small_heat3d(m=m, k=k, steps=150)
    got, ref = _compare(p)
    assert ref["roles"] == ["gen", "affine"]


@pytest.mark.parametrize("seed", [11, 12, 13])
def test_random_symmetric_all_roles(seed):
    # 5 generators + center + forcing = 7 runs, batched 4 + 2 + 1; n is not a
    # multiple of the block size (ragged tail)
    p = W.random_symmetric(n=1237, ngen=5, o=3, k=24, steps=80, seed=seed, affine=True, center=True)
    _compare(p)


def test_unsafe_verdict_and_counter_example():
    p = W.small_heat3d(m=12, k=20, steps=150)
    ref = oracle.verify(p)
    hi = ref["verdict"]["hi"]
    # the row whose reachable maximum grows most over time; unsafe threshold
    # half-way between its value at t=0 and its peak
    q = int(np.argmax(hi.max(axis=0) - hi[0]))
    assert hi[:, q].max() > hi[0, q]
    p.unsafe = np.array([[math.inf, math.inf]] * p.o)
    p.unsafe[q, 0] = 0.5 * (hi[0, q] + hi[:, q].max())
    got, ref = _compare(p)
    assert ref["verdict"]["first_step"] > 0
    assert got["verdict"]["first_step"] == ref["verdict"]["first_step"]


def test_breakdown_sine_mode_and_zero_generator():
    p = W.heat1d(steps=50)
    n = p.n
    h = 1.0 / (n + 1)
    mode = np.sin(3 * math.pi * np.arange(1, n + 1) * h)
    p.gens = [W.Generator(W.segments_from_ranges([(0, 5)], 0.0), 0.0, 1.0)]   # zero generator
    p.center = mode                                                              # an eigenvector
    p.C = [W.segments_from_ranges([(90, 111)], 1.0 / 21.0)]
    got, ref = _compare(p)
    assert [r["k_eff"] for r in got["runs"]] == [0, 1]


def test_k_larger_than_invariant_space():
    # diagonal-like system with few distinct eigenvalues: breakdown before k
    n = 64
    lam = np.repeat([-1.0, -2.5, -4.0], [20, 20, 24])
    rowptr = np.arange(n + 1, dtype=np.int64)
    p = W.Problem("diag", n, "csr", True,
                  [W.Generator(W.segments_from_ranges([(0, 64)], 1.0), 0.0, 1.0)],
                  [W.segments_from_ranges([(0, 20)], 0.05), W.segments_from_ranges([(40, 64)], 1 / 24)],
                  np.array([[0.9, math.inf], [0.9, math.inf]]), k=10, dt=0.1, steps=30,
                  rowptr=rowptr, colidx=np.arange(n, dtype=np.int32), vals=lam)
    got, ref = _compare(p)
    assert got["runs"][0]["k_eff"] == 3
    t = np.arange(31) * 0.1
    np.testing.assert_allclose(got["basis"][:, 0, 0], np.exp(-t), rtol=1e-13)


def test_stencil_matches_csr_and_oracle():
    p = W.small_heat3d(m=11, k=18, steps=60)
    ps = W.Problem("stencil", p.n, "stencil7", True, p.gens, p.C, p.unsafe, k=p.k, dt=p.dt, steps=p.steps,
                   b=p.b, grid=(11, 11, 11), coef=p.meta["coef"])
    got_s, ref = _compare(ps)
    got_c = gpu_verify(p)
    assert_basis_parity(got_s["basis"], got_c["basis"])


def test_tiny_and_degenerate_sizes():
    # n = 1, k = 1, steps = 0
    p = W.Problem("scalar", 1, "csr", True, [W.Generator(W.segments_from_ranges([(0, 1)], 2.0), 0.5, 0.1)],
                  [W.segments_from_ranges([(0, 1)])], np.array([[-math.inf, 0.5]]), k=1, dt=0.3, steps=0,
                  rowptr=np.array([0, 1], dtype=np.int64), colidx=np.array([0], dtype=np.int32),
                  vals=np.array([-0.7]))
    got, ref = _compare(p)
    np.testing.assert_allclose(got["basis"][0, 0, 0], 2.0, rtol=1e-15)
    assert got["verdict"]["first_step"] == -1
    p.steps = 7
    got, ref = _compare(p)
    np.testing.assert_allclose(got["basis"][:, 0, 0], 2.0 * np.exp(-0.7 * 0.3 * np.arange(8)), rtol=1e-14)


def test_batching_and_repeat_are_bitwise_identical():
    require_gpu()
    p = W.random_symmetric(n=3001, ngen=7, o=2, k=16, steps=40, seed=5, affine=True, center=False)
    from paper_1804_01583_amd import kry
    dsys = kry.DeviceSystem(p)
    ref = gpu_verify(p, dsys=dsys, block_p=1)["basis"]
    for bp in (2, 4, 8, 0):
        got = gpu_verify(p, dsys=dsys, block_p=bp)["basis"]
        np.testing.assert_array_equal(got, ref)
    again = gpu_verify(p, dsys=dsys, block_p=0)["basis"]
    np.testing.assert_array_equal(again, ref)


def test_workspace_from_library_allocation():
    p = W.small_heat3d(m=9, k=12, steps=20)
    require_gpu()
    a = gpu_verify(p, workspace="library")["basis"]
    b = gpu_verify(p, workspace="torch")["basis"]
    np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("block_p", [1, 2, 4, 0])
def test_marching_stencil_ragged_grid(monkeypatch, block_p):
    # the marching mat-vec (one thread per (y, z) column) on a grid whose
    # column count is not a multiple of the block, forced on at a small size
    monkeypatch.setenv("KRY_STENCIL_MARCH", "1")
    grid = (13, 17, 19)
    n = int(np.prod(grid))
    rng = np.random.default_rng(31)
    gens = [W.Generator(W.box_segments(grid, ((2 + g, 6 + g), (3, 9 + g), (1 + g, 12)), 1.0),
                        zc=0.5 * g, radius=0.2) for g in range(5)]
    C = [W.box_segments(grid, ((6, 7), (8, 9), (9, 10)), 1.0),
         W.box_segments(grid, ((0, 13), (0, 17), (0, 19)), 1.0 / n),
         W.box_segments(grid, ((10, 13), (0, 4), (15, 19)), 2.0)]
    b = np.zeros(n)
    b[rng.choice(n, 40, replace=False)] = rng.uniform(0.5, 1.5, 40)
    p = W.Problem("march", n, "stencil7", True, gens, C, np.array([[math.inf, math.inf]] * 3),
                  k=22, dt=0.05, steps=90, b=b, grid=grid, coef=(-0.9, 0.1, 0.12, 0.14))
    got, ref = _compare(p, block_p=block_p)
    monkeypatch.setenv("KRY_STENCIL_MARCH", "0")
    rows = gpu_verify(p, block_p=block_p)
    assert_basis_parity(got["basis"], rows["basis"])


def test_marching_stencil_under_arnoldi(monkeypatch):
    monkeypatch.setenv("KRY_STENCIL_MARCH", "1")
    p = W.small_heat3d(m=10, k=15, steps=50)
    ps = W.Problem("stencil", p.n, "stencil7", True, p.gens, p.C, p.unsafe, k=p.k, dt=p.dt, steps=p.steps,
                   b=p.b, grid=(10, 10, 10), coef=p.meta["coef"])
    require_gpu()
    ref = oracle.verify(ps, method="arnoldi")
    got = gpu_verify(ps, method=2)
    assert_basis_parity(got["basis"], ref["basis"])
