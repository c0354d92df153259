"""The stated configurations at their own sizes and precisions:

* the 1000^3 matrix-free heat system (10^9 states, k = 20, 500 steps) in
  FP32-basis mode, against the FP64 oracle on its locality sub-grids (each
  run equals the same run on the sub-grid of its start box dilated by
  k + 1 cells), with identical verdicts on thresholds whose FP64 margin
  exceeds the stated bound;
* block Arnoldi shaped like the 10^7 convection-diffusion configuration
  (16 generators as one p = 16 block, k = 30 block steps, 5 outputs) at
  10^6 rows, FP64 and FP32 basis, against oracle/block.py's result (stored
  under golden/, written by golden/make_block_convdiff.py);
* the dense small stage at Krylov dimension 2048 (three-vector Lanczos),
  against the oracle's per-step Pade exponential.

FP32-basis mode has no precision fixed by the paper; its stated bound is a
relative error of FP32_BOUND per (output row, basis column) against the
FP64 result (measured errors lie at 1e-9 .. 2e-5), and its verdicts must
equal the FP64 ones wherever the FP64 margin to a threshold exceeds that
bound times the row's scale."""
import math
import os

import numpy as np
import pytest
import torch  # noqa: F401

import oracle
import workloads as W
from paper_1804_01583_amd import kry
from tests.golden import make_block_convdiff
from tests.gpu_helpers import RTOL, assert_basis_parity, require_gpu
from tests.test_gpu_block import assert_block_basis_parity, gpu_block

pytestmark = pytest.mark.gpu

FP32_BOUND = 1e-4


def _rel_err(a, r):
    scale = np.abs(r).max()
    if scale == 0.0:
        assert np.all(a == 0.0)
        return 0.0
    return float(np.abs(a - r).max() / scale)


def test_heat3d_1000_fp32_basis_full_size_by_locality():
    require_gpu()
    full = W.heat3d_stencil(m=1000)
    print(f"[gpu] heat3d_stencil m=1000 FP32 basis n={full.n}", flush=True)
    # the FP64 reference basis, assembled from the oracle's sub-grid runs
    ref = np.zeros((full.steps + 1, full.o, 2))
    for r, role in enumerate(["gen", "affine"]):
        sub, rows = W.heat3d_stencil_subgrid(full, role)
        if sub is None:
            continue
        rb = oracle.verify(sub)["basis"]
        for q, c in enumerate(rows):
            if c is not None:
                ref[:, q, r] = rb[:, c, 0]
    # thresholds on the heated region's mean (row 1) whose FP64 margin at
    # every step exceeds 10x the stated bound times the row's scale: one that
    # the reachable lower end is below from step 0 on (unsafe at once) and one
    # it never reaches (safe); the mean changes too slowly per step (1e-11
    # relative) for a crossing mid-run to be decided in FP32 storage
    zc, rad = full.gens[0].zc, full.gens[0].radius
    lo = ref[:, 1, 0] * zc - abs(ref[:, 1, 0]) * rad + ref[:, 1, 1]
    scale = np.abs(ref[:, 1, :]).max()
    gap = 10 * FP32_BOUND * scale
    cases = [(lo.max() + gap, 0), (lo.min() - gap, -1)]
    plan = kry.Plan(kry.DeviceSystem(full), precision=kry.KRY_FP32_BASIS, workspace="library")
    got = plan.basis()
    v_default = plan.check(full.unsafe)
    verdicts = [plan.check(np.array([[math.inf, math.inf], [-math.inf, th]])) for th, _ in cases]
    plan.close()
    errs = [[_rel_err(got[:, q, r], ref[:, q, r]) for r in range(2)] for q in range(full.o)]
    print(f"  FP32-basis relative error per (row, column): {errs}", flush=True)
    assert max(max(e) for e in errs) <= FP32_BOUND
    want_default = oracle.box_check(ref, ["gen", "affine"], np.array([zc]), np.array([rad]), full.unsafe)
    assert v_default["first_step"] == want_default["first_step"] == -1
    for (th, first), v in zip(cases, verdicts):
        want = oracle.box_check(ref, ["gen", "affine"], np.array([zc]), np.array([rad]),
                                np.array([[math.inf, math.inf], [-math.inf, th]]))
        assert want["first_step"] == first
        assert v["first_step"] == first and (first < 0 or v["row"] == 1)


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "block_convdiff_100.npz")


@pytest.mark.parametrize("precision", [kry.KRY_FP64, kry.KRY_FP32_BASIS], ids=["fp64", "fp32"])
def test_block_arnoldi_convdiff_1e6_rows(precision):
    # 100^3 convection-diffusion, 2 random off-stencil entries per row, 16
    # generators over seeded ranges of 1000 rows as one block, k = 30; the
    # oracle's result (minutes of CPU) is stored by golden/make_block_convdiff.py
    require_gpu()
    prob = make_block_convdiff.problem()
    ref = np.load(GOLDEN)
    got = gpu_block(prob, 16, precision=precision)
    rtol = RTOL if precision == kry.KRY_FP64 else FP32_BOUND
    worst = assert_block_basis_parity(got["basis"], ref["basis"], 16, rtol=rtol)
    gv = got["verdict"]
    assert (gv["first_step"], gv["row"]) == (int(ref["first_step"]), int(ref["row"]))
    if precision == kry.KRY_FP64:
        g = got["blocks"][0]
        assert g["k_eff"] == int(ref["k_eff"]) == 30
        p = 16
        H = g["H"]
        scale = np.abs(ref["h_diag"]).max()
        for i in range(30):
            np.testing.assert_allclose(H[i * p:(i + 1) * p, i * p:(i + 1) * p], ref["h_diag"][i],
                                       rtol=0, atol=RTOL * scale)
        for i in range(29):
            np.testing.assert_allclose(H[(i + 1) * p:(i + 2) * p, i * p:(i + 1) * p], ref["h_sub"][i],
                                       rtol=0, atol=RTOL * scale)
    print(f"  block 1e6 precision={precision} worst relative error {worst:.2e}", flush=True)


def test_dense_stage_at_k_2048():
    # three-vector Lanczos of Algorithm 4 at k = 2048 on the paper's heat
    # operator (20^3 grid); the small stage is the dense one at m = 2048
    require_gpu()
    p = W.heat3d_paper(m=20, k=2048, steps=5)
    # output: the heated region's mean (the centre point stays at zero
    # within 5 steps)
    gbox = p.meta["gen_box"]
    cells = int(np.prod([b - a for a, b in gbox]))
    p.C = [W.box_segments((20, 20, 20), gbox, 1.0 / cells)]
    print(f"[gpu] dense stage k=2048 n={p.n}", flush=True)
    ref = oracle.verify(p, method="lanczos", k=2048)
    from tests.gpu_helpers import gpu_verify
    got = gpu_verify(p, method=kry.KRY_LANCZOS_PLAIN)
    assert got["runs"][0]["k_eff"] == ref["runs"][0].k_eff == 2048
    worst = assert_basis_parity(got["basis"], ref["basis"])
    print(f"  worst relative error {worst:.2e}", flush=True)
