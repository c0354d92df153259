"""CPU FP64 oracle for projected Krylov simulation and the box safety check.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, the ``smoke()`` entry and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library; both sides read the same seeded inputs from ``workloads``.

It is a plain, slow, obviously correct restatement of the paper
(Bak, Tran, Johnson, "Numerical Verification of Affine Systems with up to a
Billion Dimensions", arXiv 1804.01583):

* affine-to-linear augmentation (Section 2.1),
* output and initial-space projection, C e^{At} E (Sections 3.1, 3.2),
* basis columns by simulation from each column of E (Section 4.1),
* Arnoldi (Algorithm 1) and Lanczos with on-the-fly projection
  (Algorithms 3 and 4, fixed k) and the approximation
  e^{At} v ~ |v| V_k e^{H_k t} e_1 (Section 4.2, Eq. approx-formula),
* the small matrix exponential by Pade [13/13] scaling and squaring
  (Higham 2005), one independent exponential per time step,
* the per-step check, specialised from the LP of Section 2.1 to a box
  initial set and per-row interval unsafe sets, with a counter-example,
* block Arnoldi over p generator columns at once (``block``), the same
  Galerkin approximant for a block start,
* the a-posteriori choice of k by the error bound of Lemma 1 (``adaptive``),
* the basis by simulation of the transposed dynamics, one run per output
  row (Section 4.1, ``transpose``),
* the per-step safety LP of Section 2.1 for a polytopic initial set and a
  conjunction of output halfspaces (``lp``, SciPy's linprog as the solver).

All pins of these functions live in ``tests/test_oracle_*.py``.
"""
from .krylov import (  # noqa: F401
    BREAKDOWN_FACTOR, augment, arnoldi, lanczos, expm_pade13, pade13_coefficients,
    project_steps, build_runs, verify, box_check, system_matrix, output_matrix,
    RunResult, krylov_run,
)
from .block import BlockResult, block_arnoldi, block_project_steps, block_verify, qr_posdiag  # noqa: F401
from . import adaptive  # noqa: F401
from . import transpose  # noqa: F401
from . import lp  # noqa: F401
