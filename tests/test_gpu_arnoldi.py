"""GPU parity of the Arnoldi (CGS2) path for nonsymmetric A, including the
paper's worked example run end to end on the GPU."""
import json
import math
import os

import numpy as np
import pytest
import torch  # noqa: F401  (imported at collection so the first test does not pay for it)

import oracle
import workloads as W
from tests.gpu_helpers import (assert_basis_parity, assert_krylov_parity, assert_verdict_parity, gpu_verify,
                               require_gpu)

pytestmark = pytest.mark.gpu

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "harmonic.json")))


def _compare(problem, oracle_method="auto", **kw):
    require_gpu()
    ref = oracle.verify(problem, method=oracle_method, k=kw.get("k"), steps=kw.get("steps"), dt=kw.get("dt"))
    got = gpu_verify(problem, **kw)
    assert got["roles"] == ref["roles"]
    for g, r in zip(got["runs"], ref["runs"]):
        assert_krylov_parity(g, r)
    worst = assert_basis_parity(got["basis"], ref["basis"])
    assert_verdict_parity(got["verdict"], ref["verdict"], ref["basis"])
    print(f"  worst relative error {worst:.2e}", flush=True)
    return got, ref


def test_harmonic_oscillator_worked_example():
    # Section 2.2: unsafe at 3*pi/4 with y0 = 0.66; basis (0.707, 3.54) at that step
    p = W.harmonic_oscillator()
    got, ref = _compare(p)
    assert got["roles"] == ["gen", "center", "affine"]
    v = got["verdict"]
    assert v["first_step"] == GOLD["verdicts"]["unsafe_first_step"]
    np.testing.assert_allclose(v["z"][0], GOLD["counter_example"]["x0"][1], atol=5e-3)
    M = got["basis"][3, 0]
    np.testing.assert_allclose([M[0], M[1] + M[2]], GOLD["projected_basis_CeAtE_at_3pi_over_4"]["row"],
                               atol=5e-3)
    assert [r["k_eff"] for r in got["runs"]] == [2, 2, 2]


@pytest.mark.parametrize("grid,seed", [((12, 12, 14), 3), ((9, 11, 13), 4)])
def test_convection_diffusion(grid, seed):
    p = W.conv_diff3d(*grid, ngen=3, gen_len=40, o=3, k=20, steps=120, dt=1e-3, seed=seed)
    got, ref = _compare(p)
    assert ref["roles"] == ["gen"] * 3


def test_nonsymmetric_with_center_and_forcing():
    p = W.conv_diff3d(10, 10, 11, ngen=2, gen_len=30, o=2, k=16, steps=60, dt=2e-3, seed=8)
    rng = np.random.default_rng(8)
    p.b = rng.normal(0, 1, p.n) * (rng.uniform(size=p.n) < 0.05)
    p.center = rng.normal(0, 1, p.n) * (rng.uniform(size=p.n) < 0.05)
    got, ref = _compare(p)
    assert got["roles"] == ["gen", "gen", "center", "affine"]


def test_arnoldi_on_symmetric_matches_lanczos():
    p = W.small_heat3d(m=10, k=18, steps=80)
    got_a, ref_a = _compare(p, oracle_method="arnoldi", method=2)   # KRY_ARNOLDI
    got_l = gpu_verify(p)
    assert_basis_parity(got_a["basis"], got_l["basis"], rtol=1e-10)


def test_nilpotent_terminates_exactly():
    # down-shift: the Krylov space from e_1 is the whole space (k_eff = n)
    n = 6
    p = W.Problem("shift", n, "csr", False, [W.Generator(W.segments_from_ranges([(0, 1)]), 0.0, 1.0)],
                  [W.segments_from_ranges([(q, q + 1)]) for q in range(n)],
                  np.array([[math.inf, math.inf]] * n), k=10, dt=0.3, steps=5,
                  rowptr=np.array([0, 0, 1, 2, 3, 4, 5], dtype=np.int64),
                  colidx=np.arange(0, 5, dtype=np.int32), vals=np.ones(5))
    got, ref = _compare(p)
    assert got["runs"][0]["k_eff"] == n
    t = 5 * 0.3
    exact = np.array([t**j / math.factorial(j) for j in range(n)])
    np.testing.assert_allclose(got["basis"][5, :, 0], exact, rtol=1e-12)
