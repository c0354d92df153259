"""GPU parity of the persistent small-system kernels (FP64, at most 2048
rows: every run of a plan in one launch; Lanczos with its three vectors in
LDS, Arnoldi up to k = 64 with its basis in a per-run slice of the
workspace) against the oracle and against the general multi-launch path
(KRY_SMALL=0)."""
import math

import numpy as np
import pytest
import torch  # noqa: F401  (imported at collection so the first test does not pay for it)

import oracle
import workloads as W
from tests.gpu_helpers import (assert_basis_parity, assert_krylov_parity, assert_verdict_parity, env, gpu_verify,
                               require_gpu)

pytestmark = pytest.mark.gpu


def _both(problem, **kw):
    """The oracle, the persistent path and the general path on one problem."""
    require_gpu()
    ref = oracle.verify(problem, k=kw.get("k"), steps=kw.get("steps"), dt=kw.get("dt"))
    small = gpu_verify(problem, **kw)
    with env(KRY_SMALL="0"):
        general = gpu_verify(problem, **kw)
    assert small["roles"] == ref["roles"] == general["roles"]
    for g, r in zip(small["runs"], ref["runs"]):
        assert_krylov_parity(g, r)
    worst = assert_basis_parity(small["basis"], ref["basis"])
    assert_verdict_parity(small["verdict"], ref["verdict"], ref["basis"])
    d = assert_basis_parity(small["basis"], general["basis"], rtol=1e-12)
    assert [r["k_eff"] for r in small["runs"]] == [r["k_eff"] for r in general["runs"]]
    print(f"  worst relative error {worst:.2e}, against the general path {d:.2e}", flush=True)
    return small, general, ref


def test_heat1d_ten_generators():
    # the 1D heat configuration: n = 200, ten generators, k = 30, 1000 steps
    small, _, _ = _both(W.heat1d())
    assert small["roles"] == ["gen"] * 10


def test_random_symmetric_with_center_and_forcing():
    p = W.random_symmetric(n=400, k=16, steps=80, ngen=4, o=3, affine=True, center=True)
    small, _, _ = _both(p)
    assert small["roles"] == ["gen"] * 4 + ["center", "affine"]


def test_stencil_with_forcing():
    p = W.small_heat3d(m=11, k=18, steps=60)
    ps = W.Problem("stencil", p.n, "stencil7", True, p.gens, p.C, p.unsafe, k=p.k, dt=p.dt, steps=p.steps,
                   b=p.b, grid=(11, 11, 11), coef=p.meta["coef"])
    _both(ps)


def test_largest_small_size_and_the_next():
    # 2048 rows take the persistent kernel, 2049 the general path
    for n in (2048, 2049):
        p = W.random_symmetric(n=n, k=12, steps=40, ngen=3, o=2, affine=False)
        _both(p)


def test_more_runs_than_one_launch():
    # 70 generators: two launches of the persistent kernel (64 + 6 runs)
    p = W.heat1d(n=300, k=10, steps=50)
    rng = np.random.default_rng(3)
    p.gens = [W.Generator(W.segments_from_ranges([(j, j + 3)]), zc=float(rng.uniform()), radius=0.05)
              for j in range(0, 210, 3)]
    small, _, _ = _both(p)
    assert len(small["runs"]) == 70


def test_breakdown_on_an_eigenvector():
    # a Dirichlet sine mode: the Krylov space is one-dimensional
    p = W.heat1d(n=120, k=6, steps=30)
    n = p.n
    x = np.arange(1, n + 1) / (n + 1)
    v = np.sin(3 * math.pi * x)
    p.gens = [W.Generator(W.Segments(np.arange(n), np.arange(n) + 1, v), zc=1.0, radius=0.1)]
    p.unsafe = np.array([[math.inf, math.inf]])
    small, general, _ = _both(p)
    assert small["runs"][0]["k_eff"] == 1 == general["runs"][0]["k_eff"]
    lam = -4 * (n + 1) ** 2 * math.sin(3 * math.pi / (2 * (n + 1))) ** 2
    t = np.arange(p.steps + 1) * p.dt
    want = oracle.output_matrix(p).toarray() @ v
    np.testing.assert_allclose(small["basis"][:, 0, 0], want[0] * np.exp(lam * t), rtol=1e-12)


def test_arnoldi_convection_diffusion():
    p = W.conv_diff3d(12, 12, 14, ngen=3, gen_len=40, o=3, k=20, steps=120, dt=1e-3, seed=3)
    small, _, _ = _both(p)
    assert small["roles"] == ["gen"] * 3


def test_arnoldi_with_center_and_forcing():
    p = W.conv_diff3d(10, 10, 11, ngen=2, gen_len=30, o=2, k=16, steps=60, dt=2e-3, seed=8)
    rng = np.random.default_rng(8)
    p.b = rng.normal(0, 1, p.n) * (rng.uniform(size=p.n) < 0.05)
    p.center = rng.normal(0, 1, p.n) * (rng.uniform(size=p.n) < 0.05)
    small, _, _ = _both(p)
    assert small["roles"] == ["gen", "gen", "center", "affine"]


def test_arnoldi_nilpotent_terminates_exactly():
    # down-shift: the Krylov space from e_1 is the whole space (k_eff = n)
    n = 6
    p = W.Problem("shift", n, "csr", False, [W.Generator(W.segments_from_ranges([(0, 1)]), 0.0, 1.0)],
                  [W.segments_from_ranges([(q, q + 1)]) for q in range(n)],
                  np.array([[math.inf, math.inf]] * n), k=10, dt=0.3, steps=5,
                  rowptr=np.array([0, 0, 1, 2, 3, 4, 5], dtype=np.int64),
                  colidx=np.arange(0, 5, dtype=np.int32), vals=np.ones(5))
    small, _, _ = _both(p)
    assert small["runs"][0]["k_eff"] == n
    t = 5 * 0.3
    exact = np.array([t**j / math.factorial(j) for j in range(n)])
    np.testing.assert_allclose(small["basis"][5, :, 0], exact, rtol=1e-12)


def test_arnoldi_past_the_small_kernels_k():
    # k = 65 > 64: the general path, and its result
    p = W.conv_diff3d(9, 10, 11, ngen=1, gen_len=40, o=2, k=65, steps=40, dt=1e-3, seed=2)
    _both(p)
