"""GPU parity of block Arnoldi (KRY_BLOCK_ARNOLDI) against the block oracle
(oracle/block.py): the basis C V e^{H s dt} E_1 R_0 and H, R_0, P per block
run (unique, since both sides use a non-negative diag(R)), within 1e-10.

The basis bound is relative to the block's scale on each output row,
max over steps and over the block's generator columns, not to each column's
own scale: the columns of a block share one basis, so a column whose output
on a row is far smaller than another column's is formed by cancellation at
the larger scale, and both sides can only resolve it to eps times that
scale."""
import math

import numpy as np
import pytest
import torch  # noqa: F401  (imported at collection so the first test does not pay for it)

import oracle
import workloads as W
from oracle import block as OB
from paper_1804_01583_amd import kry
from tests.gpu_helpers import RTOL, assert_basis_parity, env, gpu_verify, require_gpu

pytestmark = pytest.mark.gpu


def gpu_block(problem, p, precision=kry.KRY_FP64, k=None, steps=None):
    require_gpu()
    print(f"[gpu] block {problem.name} n={problem.n} p={p} k={k or problem.k} steps={steps or problem.steps} "
          f"precision={precision}", flush=True)
    dsys = kry.DeviceSystem(problem)
    plan = kry.Plan(dsys, k=k, steps=steps, method=kry.KRY_BLOCK_ARNOLDI, block_p=p, precision=precision)
    basis = plan.basis()
    verdict = plan.check(problem.unsafe)
    blocks = plan.blocks()
    plan.close()
    return {"basis": basis, "verdict": verdict, "blocks": blocks}


def assert_block_basis_parity(got, ref, p, rtol=RTOL):
    """max_s,c |y_gpu - y_ref| <= rtol * max_s,c |y_ref| over the columns c of
    each block, per output row; rows the oracle gives as zero stay zero."""
    assert got.shape == ref.shape
    S1, o, ng = ref.shape
    worst = 0.0
    for b0 in range(0, ng, p):
        for q in range(o):
            a, r = got[:, q, b0:b0 + p], ref[:, q, b0:b0 + p]
            scale = np.abs(r).max()
            if scale == 0.0:
                assert np.all(a == 0.0)
                continue
            err = np.abs(a - r).max() / scale
            worst = max(worst, err)
            assert err <= rtol, f"block {b0 // p} row {q}: relative error {err:.3e} > {rtol:.1e}"
    return worst


def _compare_blocks(got, ref, rtol=RTOL):
    assert len(got["blocks"]) == len(ref["blocks"])
    for g, r in zip(got["blocks"], ref["blocks"]):
        assert g["k_eff"] == r.k_eff and g["p"] == r.p
        np.testing.assert_allclose(g["R0"], r.R0, rtol=0, atol=rtol * np.abs(r.R0).max())
        np.testing.assert_allclose(g["H"], r.H, rtol=0, atol=rtol * np.abs(r.H).max())
        ps = np.abs(r.P).max()
        np.testing.assert_allclose(g["P"], r.P, rtol=0, atol=rtol * max(ps, 1e-300))


@pytest.mark.parametrize("grid,ngen,p,k", [((9, 10, 11), 5, 3, 6), ((12, 12, 14), 16, 16, 4),
                                           ((8, 9, 10), 7, 4, 9)])
def test_block_matches_oracle(grid, ngen, p, k):
    prob = W.conv_diff3d(*grid, ngen=ngen, gen_len=6, o=3, k=k, steps=60, dt=2e-3, seed=11)
    ref = OB.block_verify(prob, p=p)
    got = gpu_block(prob, p)
    _compare_blocks(got, ref)
    worst = assert_block_basis_parity(got["basis"], ref["basis"], p)
    gv, ov = got["verdict"], ref["verdict"]
    assert (gv["first_step"], gv["row"]) == (ov["first_step"], ov["row"])
    print(f"  worst relative error {worst:.2e}", flush=True)


def test_block_p1_equals_single_vector_arnoldi():
    prob = W.conv_diff3d(9, 9, 10, ngen=2, gen_len=8, o=2, k=12, steps=40, dt=2e-3, seed=5)
    got = gpu_block(prob, 1)
    single = gpu_verify(prob, method=kry.KRY_ARNOLDI)
    assert_basis_parity(got["basis"], single["basis"])


def test_block_largest_dimension():
    # k = 32 block steps of 16 columns: the dense stage at m = 512
    prob = W.conv_diff3d(20, 20, 25, ngen=16, gen_len=20, o=2, k=32, steps=12, dt=1e-3, seed=4)
    ref = OB.block_verify(prob, p=16)
    got = gpu_block(prob, 16)
    _compare_blocks(got, ref)
    assert_block_basis_parity(got["basis"], ref["basis"], 16)


def test_block_breakdown_on_eigenvector_block():
    # two Dirichlet sine modes span an invariant space: one block step, exact
    prob = W.heat1d(n=120, k=4, steps=30)
    n = prob.n
    x = np.arange(1, n + 1) / (n + 1)
    gens = []
    for mode in (2, 5):
        v = np.sin(mode * math.pi * x)
        gens.append(W.Generator(W.Segments(np.arange(n), np.arange(n) + 1, v), zc=1.0, radius=0.1))
    prob.gens = gens
    prob.C = [W.segments_from_ranges([(30, 50)], 0.05), W.segments_from_ranges([(70, 71)], 1.0)]
    prob.unsafe = np.array([[math.inf, math.inf]] * 2)
    ref = OB.block_verify(prob, p=2)
    got = gpu_block(prob, 2)
    assert got["blocks"][0]["k_eff"] == 1 == ref["blocks"][0].k_eff
    assert_block_basis_parity(got["basis"], ref["basis"], 2)
    lam = np.array([-4 * (n + 1) ** 2 * math.sin(j * math.pi / (2 * (n + 1))) ** 2 for j in (2, 5)])
    t = np.arange(prob.steps + 1) * prob.dt
    C = oracle.output_matrix(prob).toarray()
    G = np.stack([g.seg.dense(n) for g in gens], axis=1)
    want = np.einsum("qn,nc,sc->sqc", C, G, np.exp(np.outer(t, lam)))
    np.testing.assert_allclose(got["basis"], want, rtol=0, atol=1e-11 * np.abs(want).max())


def test_block_dependent_generators_are_reported():
    require_gpu()
    prob = W.conv_diff3d(8, 8, 9, ngen=3, gen_len=6, o=1, k=3, steps=5, dt=1e-3, seed=2)
    prob.gens = [prob.gens[0], prob.gens[1], prob.gens[0]]
    with pytest.raises(kry.KryError) as ei:
        gpu_block(prob, 3)
    assert ei.value.args[0].startswith(f"kry status {kry.KRY_ENUMERIC}")


def test_block_fp32_basis():
    prob = W.conv_diff3d(12, 12, 14, ngen=16, gen_len=6, o=3, k=5, steps=80, dt=2e-3, seed=13)
    ref = OB.block_verify(prob, p=16)
    got = gpu_block(prob, 16, precision=kry.KRY_FP32_BASIS)
    anorm = oracle.krylov.inf_norm(oracle.system_matrix(prob))
    tol = min(1e-4, max(1e-5, 2.0 * 2.0 ** -23 * anorm * prob.steps * prob.dt))
    worst = assert_block_basis_parity(got["basis"], ref["basis"], 16, rtol=tol)
    print(f"  FP32-basis block worst relative error {worst:.2e} (bound {tol:.1e})", flush=True)


def test_block_rejects_center_and_forcing():
    require_gpu()
    prob = W.small_heat3d(m=6, k=4, steps=5)
    with pytest.raises(kry.KryError) as ei:
        gpu_block(prob, 1)
    assert ei.value.args[0].startswith(f"kry status {kry.KRY_ENOTSUP}")


@pytest.mark.parametrize("precision", [kry.KRY_FP64, kry.KRY_FP32_BASIS])
def test_block_gram_corrected_pass_against_two_passes(precision):
    # the second Gram-Schmidt pass from the Gram matrix of the stored blocks
    # against the plain second pass over the basis, and both against the oracle
    prob = W.conv_diff3d(12, 12, 14, ngen=16, gen_len=6, o=3, k=10, steps=60, dt=2e-3, seed=11)
    ref = OB.block_verify(prob, p=16)
    with env(KRY_BLOCK_GS="0"):
        two = gpu_block(prob, 16, precision=precision)
    one = gpu_block(prob, 16, precision=precision)
    if precision == kry.KRY_FP64:
        _compare_blocks(one, ref)
        assert_block_basis_parity(one["basis"], ref["basis"], 16)
        d = assert_block_basis_parity(one["basis"], two["basis"], 16, rtol=1e-12)
    else:
        anorm = oracle.krylov.inf_norm(oracle.system_matrix(prob))
        tol = min(1e-4, max(1e-5, 2.0 * 2.0 ** -23 * anorm * prob.steps * prob.dt))
        assert_block_basis_parity(one["basis"], ref["basis"], 16, rtol=tol)
        d = assert_block_basis_parity(one["basis"], two["basis"], 16, rtol=tol)
    print(f"  one-pass against two-pass: {d:.2e}", flush=True)


def _near_invariant_problem():
    # two Dirichlet sine modes plus 5e-6 of a local bump each: the first block
    # step keeps 8e-5 and 5e-4 of |A V_1| after the projection (far above
    # breakdown, and far enough that the later directions, which come from
    # the bumps, are fixed to ~1e-12 by the data)
    prob = W.heat1d(n=120, k=6, steps=30)
    n = prob.n
    x = np.arange(1, n + 1) / (n + 1)
    gens = []
    for mode, (a, b) in ((2, (40, 51)), (5, (70, 76))):
        v = np.sin(mode * math.pi * x)
        v[a:b] += 5e-6
        gens.append(W.Generator(W.Segments(np.arange(n), np.arange(n) + 1, v), zc=1.0, radius=0.1))
    prob.gens = gens
    prob.C = [W.segments_from_ranges([(30, 50)], 0.05), W.segments_from_ranges([(70, 71)], 1.0)]
    prob.unsafe = np.array([[math.inf, math.inf]] * 2)
    return prob


def test_block_second_pass_when_the_projection_cancels():
    prob = _near_invariant_problem()
    ref = OB.block_verify(prob, p=2)
    got = gpu_block(prob, 2)
    _compare_blocks(got, ref)
    assert_block_basis_parity(got["basis"], ref["basis"], 2)
    # the plain second pass ran: it adds its (tiny) coefficients to H, so
    # without it H differs (the outputs, dominated by the sine modes, may not)
    with env(KRY_BLOCK_REORTH2="0"):
        nopass = gpu_block(prob, 2)
    assert not np.array_equal(got["blocks"][0]["H"], nopass["blocks"][0]["H"])
    # the conditional launches give the oracle's result when forced every step
    with env(KRY_BLOCK_REORTH2="1e300"):
        always = gpu_block(prob, 2)
    _compare_blocks(always, ref)
    assert_block_basis_parity(always["basis"], ref["basis"], 2)
