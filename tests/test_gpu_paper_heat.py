"""The paper's 3D heat benchmark on the GPU: stencil face conditions
(insulated faces, exchange through x = 1) in the row-form and marching
stencil kernels against the oracle's CSR expansion and against the CSR form
of the same operator."""
import dataclasses
import os

import pytest
import torch  # noqa: F401  (imported at collection so the first test does not pay for it)

import oracle
import workloads as W
from tests.gpu_helpers import assert_basis_parity, assert_verdict_parity, gpu_verify, require_gpu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("march", ["0", "1"])
def test_insulated_stencil_matches_oracle_and_csr(march):
    require_gpu()
    s = W.heat3d_paper_stencil(m=14, k=40, steps=200)
    c = W.heat3d_paper(m=14, k=40, steps=200)
    old = os.environ.get("KRY_STENCIL_MARCH")
    os.environ["KRY_STENCIL_MARCH"] = march
    try:
        got = gpu_verify(s)
    finally:
        if old is None:
            del os.environ["KRY_STENCIL_MARCH"]
        else:
            os.environ["KRY_STENCIL_MARCH"] = old
    ref = oracle.verify(s)
    worst = assert_basis_parity(got["basis"], ref["basis"])
    assert_verdict_parity(got["verdict"], ref["verdict"], ref["basis"])
    assert_basis_parity(got["basis"], gpu_verify(c)["basis"])
    print(f"  march={march} worst {worst:.2e}", flush=True)


def test_dirichlet_stencil_with_exchange_face():
    require_gpu()
    p = W.heat3d_stencil(m=12, k=30, dt=0.01, steps=100)
    p = dataclasses.replace(p, exchange=-0.3 * p.coef[1])
    got = gpu_verify(p)
    ref = oracle.verify(p)
    assert_basis_parity(got["basis"], ref["basis"])
