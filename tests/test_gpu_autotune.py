"""The launch-choice tuner (kry_plan_autotune): it stores a choice per
device, kernel and shape, later plans use it, and every choice gives the
same basis bit for bit (block mat-vec rows per workgroup and their order;
plain or non-temporal stores of the marching one-pass step)."""
import os

import numpy as np
import pytest
import torch  # noqa: F401

import workloads as W
from paper_1804_01583_amd import kry
from tests.gpu_helpers import require_gpu
from tests.test_gpu_onepass import env

pytestmark = pytest.mark.gpu


def _basis(p, **kw):
    plan = kry.Plan(kry.DeviceSystem(p), **kw)
    b = plan.basis()
    v = plan.check(p.unsafe)
    plan.close()
    return b, v


def _with_choice(path, line_of, kernel, n, runs, a, b):
    """Rewrite the cache file so that (kernel, n, runs) holds (a, b)."""
    tag = line_of.split()[0]
    path.write_text(f"{tag} {kernel} {n} {runs} {a} {b} 1.0\n")
    kry.kry_tune_clear()
    assert kry.kry_tune_choice(kernel, n, runs)[:2] == (a, b)


def test_block_spmm_choices_leave_the_basis_unchanged(tmp_path):
    require_gpu()
    p = W.conv_diff3d(20, 20, 25, ngen=16, gen_len=50, o=3, k=8, steps=40, dt=1e-4)
    path = tmp_path / "tune.txt"
    with env(KRY_TUNE_CACHE=str(path)):
        kry.kry_tune_clear()
        ref, vref = _basis(p, method=kry.KRY_BLOCK_ARNOLDI, block_p=16)
        plan = kry.Plan(kry.DeviceSystem(p), method=kry.KRY_BLOCK_ARNOLDI, block_p=16)
        assert plan.autotune(reps=2) == 1
        tuned = plan.basis()
        plan.close()
        choice = kry.kry_tune_choice("bspmm", p.n, 16)
        print(f"[gpu] block spmm choice {choice}", flush=True)
        assert choice is not None and choice[0] in (32, 64, 128, 256, 512) and choice[1] in (0, 1)
        assert np.array_equal(tuned, ref)
        line = path.read_text().splitlines()[0]
        for rows, xcd in ((32, 1), (512, 0), (128, 1)):
            _with_choice(path, line, "bspmm", p.n, 16, rows, xcd)
            got, v = _basis(p, method=kry.KRY_BLOCK_ARNOLDI, block_p=16)
            assert np.array_equal(got, ref), (rows, xcd)
            assert (v["first_step"], v["row"]) == (vref["first_step"], vref["row"])
    kry.kry_tune_clear()


def test_march_store_choice_leaves_the_basis_unchanged(tmp_path):
    require_gpu()
    grid = (9, 35, 130)
    nx, ny, nz = grid
    n = nx * ny * nz
    h = 1.0 / (max(grid) + 1)
    c = 0.01 / h**2
    gen = W.box_segments(grid, ((0, 4), (2, 7), (3, 9)), 1.0)
    fb = W.box_segments(grid, ((nx - 5, nx - 1), (ny - 6, ny - 2), (1, 5)), 0.1)
    C = [W.box_segments(grid, ((1, 6), (2, 8), (2, 12)), 1.0 / 300)]
    p = W.Problem("march", n, "stencil7", True, [W.Generator(gen, zc=1.0, radius=0.1)], C,
                  np.array([[0.4, np.inf]]), k=18, dt=0.01, steps=70, b_seg=fb, grid=grid, coef=(-6 * c, c, c, c))
    path = tmp_path / "tune.txt"
    with env(KRY_STENCIL_MARCH=1, KRY_TUNE_CACHE=str(path)):
        kry.kry_tune_clear()
        ref, _ = _basis(p)
        plan = kry.Plan(kry.DeviceSystem(p))
        assert plan.autotune(reps=2) == 1
        plan.close()
        choice = kry.kry_tune_choice("lz1_march", n, 2)
        print(f"[gpu] march store choice {choice}", flush=True)
        assert choice is not None and choice[0] in (0, 1)
        line = path.read_text().splitlines()[0]
        for nt in (0, 1):
            _with_choice(path, line, "lz1_march", n, 2, nt, 0)
            got, _ = _basis(p)
            assert np.array_equal(got, ref), nt
    kry.kry_tune_clear()


def test_plans_without_a_tuned_kernel_tune_nothing():
    require_gpu()
    p = W.small_heat3d(m=10, k=12, steps=20)
    plan = kry.Plan(kry.DeviceSystem(p))
    assert plan.autotune(reps=1) == 0
    plan.close()
