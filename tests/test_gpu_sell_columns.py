"""The sliced-ELL copy stores column - row in 16 bits when every column lies
within 32767 of its row, else 32-bit columns.  Both layouts give the same
basis bit for bit (the same columns are read in the same order), prepared
or built per plan; a matrix with far columns takes the 32-bit layout and
matches the oracle."""
import os

import numpy as np
import pytest

import oracle
import workloads as W
from gpu_helpers import assert_basis_parity, assert_verdict_parity, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _general_path(monkeypatch):
    # these kernels belong to the general path: small systems would take the
    # persistent small-system kernel instead
    monkeypatch.setenv("KRY_SMALL", "0")


def _basis(p, prepared, narrow):
    from paper_1804_01583_amd import kry
    print(f"[gpu] sell columns {p.name} n={p.n} prepared={prepared} narrow={narrow}", flush=True)
    old = os.environ.get("KRY_SELL_NARROW")
    os.environ["KRY_SELL_NARROW"] = "1" if narrow else "0"
    try:
        ds = kry.DeviceSystem(p)
        if prepared:
            ds.prepare()
        plan = kry.Plan(ds, workspace="library")
        b = plan.basis()
        v = plan.check(p.unsafe)
        plan.close()
        ds.close()
    finally:
        if old is None:
            del os.environ["KRY_SELL_NARROW"]
        else:
            os.environ["KRY_SELL_NARROW"] = old
    return b, v


@pytest.mark.parametrize("prepared", [False, True])
def test_narrow_and_wide_columns_agree_bitwise(prepared):
    require_gpu()
    p = W.heat3d_csr(m=40, k=20, steps=200)      # columns within 1600 of their rows
    b16, v16 = _basis(p, prepared, True)
    b32, v32 = _basis(p, prepared, False)
    assert np.array_equal(b16, b32)
    assert v16["first_step"] == v32["first_step"]


def _far_symmetric(n=70000, seed=3):
    """A symmetric negative definite matrix whose rows also couple to rows
    33000 to 36000 away (columns outside 16 bits of the row), with two
    generators, two output rows and a forcing."""
    import math
    import scipy.sparse as sp
    rng = np.random.default_rng(seed)
    a = rng.integers(0, n - 36000, size=n // 8)
    b = a + rng.integers(33000, 36000, size=a.size)
    far = sp.coo_matrix((np.full(a.size, 0.3), (a, b)), shape=(n, n))
    far = far + far.T
    lap = sp.diags([np.ones(n - 1), np.ones(n - 1)], [-1, 1])
    A = (lap + far).tocsr()
    A = A - sp.diags(np.asarray(abs(A).sum(axis=1)).ravel() + 0.5)
    A = A.tocsr(); A.sum_duplicates(); A.sort_indices()
    gens = [W.Generator(W.segments_from_ranges([(100, 140)], 1.0), 0.5, 0.2),
            W.Generator(W.segments_from_ranges([(50000, 50010)], 2.0), -0.3, 0.1)]
    C = [W.segments_from_ranges([(90, 150)], 1.0 / 60), W.segments_from_ranges([(49990, 50030)], 1.0 / 40)]
    unsafe = np.array([[0.4, math.inf], [0.5, math.inf]])
    bvec = np.zeros(n); bvec[20000:20100] = 0.05
    return W.Problem("far_symmetric", n, "csr", True, gens, C, unsafe, k=14, dt=0.05, steps=60, b=bvec,
                     rowptr=A.indptr.astype(np.int64), colidx=A.indices.astype(np.int32),
                     vals=A.data.astype(np.float64), seed=seed)


def test_far_columns_take_32_bits_and_match_the_oracle():
    require_gpu()
    from gpu_helpers import gpu_verify
    p = _far_symmetric()
    assert np.abs(p.colidx.astype(np.int64) - np.repeat(np.arange(p.n), np.diff(p.rowptr))).max() > 32767
    got = gpu_verify(p)
    ref = oracle.verify(p)
    assert_basis_parity(got["basis"], ref["basis"])
    assert_verdict_parity(got["verdict"], ref["verdict"], ref["basis"])
