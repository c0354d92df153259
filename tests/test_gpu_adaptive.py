"""Error-controlled Krylov dimension on the GPU (paper Section 4.2, Lemma 1;
the checkpoints of Algorithms 2 and 4) against the oracle's adaptive
Lanczos and Arnoldi: every run stops at the same dimension with the same
bound, and the basis agrees to the FP64 parity bound.

A stop decision compares a computed bound with the target, so a case is
only meaningful when no checkpoint's bound lies within rounding of it; each
case first checks that margin on the oracle's side."""
import math

import numpy as np
import pytest
import torch  # noqa: F401  (imported at collection so the first test does not pay for it)

import workloads as W
from oracle import adaptive as AD
from paper_1804_01583_amd import kry
from tests.gpu_helpers import assert_basis_parity, env, require_gpu

pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps
MARGIN = 1e-4          # no checkpoint's bound within this fraction of the target


def _checkpoint_bounds(run, tau, lam):
    """The oracle's bound at every checkpoint the run passed."""
    H = run["H"]
    out = []
    for k in AD.k_schedule(4, H.shape[0] - 1):
        out.append(AD.lemma1_bound(H[:k, :k], H[k, k - 1], tau, lam, run["affine"]))
    if run["k_eff"] == run["k_stop"] and run["bound"] not in (0.0, math.inf):
        out.append(run["bound"])
    return out


def _bound_tol(run, tau, lam):
    """Both sides evaluate (e^{tT})_{k,1} with an absolute error of a few k
    eps times max over the eigenvalues of e^{theta t} <= e^{max(lambda,0) t}
    (both as sums of k exponentials from eigen-decompositions of T: the GPU's
    own, the oracle's LAPACK tridiagonal solver),
    so the integrals can differ by up to that times int_0^tau w(t) dt
    (tau, or tau^2 / 2 for the augmented run), scaled like the bound (of
    the normalised process)."""
    k = run["k_stop"]
    lp = max(lam, 0.0)
    wint = tau * tau / 2 if run["affine"] else tau
    return 1e-9 * run["bound"] + run["h"] * math.exp(2 * lp * tau) * 4 * k * EPS * wint


def _hess_tol(run, tau, lam):
    """Arnoldi: the GPU forms (e^{tH})_{k,1} from a Taylor polynomial and up
    to 40 doublings of e^{tH} - I, the oracle from one Pade exponential per
    node.  Both are accurate to a few eps relative to |e^{tH}|, which the
    runs here keep near e^{max(lambda,0) t}; the doublings add at most one
    rounding each."""
    k = run["k_stop"]
    lp = max(lam, 0.0)
    wint = tau * tau / 2 if run["affine"] else tau
    return 1e-8 * run["bound"] + run["h"] * math.exp(2 * lp * tau) * 4 * (k + 40) * EPS * wint


def _run(p, eps, **kw):
    print(f"[gpu] adaptive {p.name} n={p.n} k={kw.get('k', p.k)} eps={eps:g} kw={kw}", flush=True)
    arnoldi = kw.get("method") == kry.KRY_ARNOLDI
    ref = AD.adaptive_verify(p, eps=eps, kmax=kw.get("k", p.k), method="arnoldi" if arnoldi else "auto")
    tol = _hess_tol if arnoldi else _bound_tol
    tau = p.steps * p.dt
    for r in ref["runs"]:
        for b in _checkpoint_bounds(r, tau, ref["lam"]):
            assert abs(b - eps) > MARGIN * eps, f"bound {b:.6e} too close to the target {eps:g}"
    plan = kry.Plan(kry.DeviceSystem(p), **kw)
    plan.set_error_target(eps)
    basis = plan.basis()
    errs = [plan.error(r) for r in range(plan.nruns)]
    dims = [plan.krylov(r)["k_eff"] for r in range(plan.nruns)]
    verdict = plan.check(p.unsafe)
    plan.close()
    for (k_used, bound), dim, r in zip(errs, dims, ref["runs"]):
        assert k_used == r["k_stop"], (k_used, r["k_stop"])
        assert dim == r["dim"]
        if r["bound"] == math.inf:
            assert bound == -1.0           # no checkpoint reached
        elif r["bound"] == 0.0:
            assert bound == 0.0
        else:
            print(f"  bound {bound:.15e} oracle {r['bound']:.15e} diff {abs(bound - r['bound']):.2e} "
                  f"tol {tol(r, tau, ref['lam']):.2e}", flush=True)
            assert abs(bound - r["bound"]) <= tol(r, tau, ref["lam"]), (bound, r["bound"])
    worst = assert_basis_parity(basis, ref["basis"])
    print(f"  k_stop {[e[0] for e in errs]} bounds {['%.3e' % e[1] for e in errs]} worst {worst:.2e}",
          flush=True)
    assert verdict["first_step"] == ref["verdict"]["first_step"]
    return errs, ref


@pytest.mark.parametrize("eps", [1e-6, 1e-9])
def test_heat3d_csr_generator_and_forcing(eps):
    require_gpu()
    p = W.small_heat3d(m=10, k=56, steps=100)
    errs, _ = _run(p, eps)
    assert max(e[0] for e in errs) < 56


def test_heat3d_stencil():
    require_gpu()
    p = W.heat3d_stencil(m=12, k=40, dt=0.01, steps=60)
    _run(p, 1e-6)


def test_positive_eigenvalues_and_batched_runs():
    # a diagonal shift makes lambda_max > 0, so the factor e^{lambda tau} enters
    require_gpu()
    p = W.random_symmetric(n=400, ngen=6, o=2, k=40, steps=50, dt=0.05, seed=21, affine=True, center=True)
    diag = p.colidx == np.repeat(np.arange(p.n), np.diff(p.rowptr))
    p.vals = p.vals + 1.2 * diag
    errs, ref = _run(p, 1e-7)
    assert ref["lam"] > 0.0


def test_target_not_reached_keeps_k():
    require_gpu()
    p = W.small_heat3d(m=10, k=12, steps=50)
    errs, _ = _run(p, 1e-30)
    assert [e[0] for e in errs] == [12, 11]


def test_breakdown_before_first_checkpoint():
    require_gpu()
    n = 64
    lam = np.repeat([-1.0, -2.5, -4.0], [20, 20, 24])
    p = W.Problem("diag", n, "csr", True,
                  [W.Generator(W.segments_from_ranges([(0, 64)], 1.0), 0.0, 1.0)],
                  [W.segments_from_ranges([(0, 20)], 0.05), W.segments_from_ranges([(40, 64)], 1 / 24)],
                  np.array([[0.9, math.inf], [0.9, math.inf]]), k=10, dt=0.1, steps=30,
                  rowptr=np.arange(n + 1, dtype=np.int64), colidx=np.arange(n, dtype=np.int32), vals=lam)
    errs, _ = _run(p, 1e-8)
    assert errs == [(3, 0.0)]


def test_stored_basis_lanczos_beyond_lds_size():
    # k > 56 keeps the Lanczos basis and reorthogonalises; T's diagonal then
    # comes from the Hessenberg store
    require_gpu()
    p = W.random_symmetric(n=2500, ngen=3, o=3, k=90, steps=60, dt=0.02, seed=17, affine=True, center=True)
    _run(p, 1e-11)


def test_zero_target_is_off():
    require_gpu()
    p = W.small_heat3d(m=10, k=20, steps=40)
    ds = kry.DeviceSystem(p)
    a = kry.Plan(ds)
    base = a.basis()
    a.close()
    b = kry.Plan(ds)
    b.set_error_target(0.0)
    again = b.basis()
    assert [b.error(r) for r in range(b.nruns)] == [(20, -1.0), (19, -1.0)]
    b.close()
    assert np.array_equal(base, again)


def test_arnoldi_rejects_k_past_lds():
    require_gpu()
    p = W.small_heat3d(m=8, k=60, steps=10)
    plan = kry.Plan(kry.DeviceSystem(p), method=kry.KRY_ARNOLDI)
    with pytest.raises(kry.KryError) as ei:
        plan.set_error_target(1e-6)
    assert ei.value.status == kry.KRY_ENOTSUP
    plan.close()
    # block Arnoldi has no error control
    q = W.conv_diff3d(6, 6, 6, ngen=2, gen_len=20, o=2, k=8, steps=10, dt=1e-3)
    plan = kry.Plan(kry.DeviceSystem(q), method=kry.KRY_BLOCK_ARNOLDI, block_p=2)
    with pytest.raises(kry.KryError) as ei:
        plan.set_error_target(1e-6)
    assert ei.value.status == kry.KRY_ENOTSUP
    plan.close()


# ---------------------------------------------------------------------------
# Algorithm 2: Arnoldi runs (upper Hessenberg H)
# ---------------------------------------------------------------------------

def _conv_diff(shift=0.0, forcing=False, center=False):
    p = W.conv_diff3d(10, 10, 10, ngen=2, gen_len=50, o=3, k=40, steps=100, dt=1e-3, seed=5)
    if shift:
        diag = p.colidx == np.repeat(np.arange(p.n), np.diff(p.rowptr))
        p.vals = p.vals + shift * diag
    rng = np.random.default_rng(77)
    if forcing:
        p.b = rng.uniform(0.0, 1.0, p.n)
    if center:
        p.center = rng.uniform(-0.5, 0.5, p.n)
    return p


# gs: the plain two-pass Gram-Schmidt these sizes take by default, and the
# second pass from the Gram matrix (forced on here; the default from 2^16 rows)
@pytest.mark.parametrize("gs", ["0", "1"])
@pytest.mark.parametrize("eps", [1e-6, 1e-9])
def test_arnoldi_nonsymmetric(eps, gs):
    require_gpu()
    with env(KRY_ARN_GS=gs):
        errs, _ = _run(_conv_diff(), eps, method=kry.KRY_ARNOLDI)
    assert all(4 <= e[0] < 40 for e in errs)


@pytest.mark.parametrize("gs", ["0", "1"])
def test_arnoldi_forcing_center_and_positive_lambda(gs):
    # a diagonal shift past the Gershgorin radius makes lambda > 0; the
    # augmented run integrates its bound; a dense center adds a run
    require_gpu()
    p = _conv_diff(shift=0.5 * 1.0 / (1.0 / 11) / 5.0, forcing=True, center=True)
    with env(KRY_ARN_GS=gs):
        errs, ref = _run(p, 1e-7, method=kry.KRY_ARNOLDI)
    assert ref["lam"] > 0.0 and len(errs) == 4


def test_arnoldi_on_a_symmetric_system_stops_with_lanczos():
    require_gpu()
    p = W.small_heat3d(m=10, k=50, steps=100)
    ea, _ = _run(p, 1e-8, method=kry.KRY_ARNOLDI)
    el, _ = _run(p, 1e-8)
    assert [e[0] for e in ea] == [e[0] for e in el]
    for (_, a), (_, b) in zip(ea, el):
        assert abs(a - b) <= 1e-6 * b


# ---------------------------------------------------------------------------
# Large Krylov dimensions: the parallel eigen-solve (bisection, twisted
# factorisation) that checkpoints past 128 take
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("case", ["heat3d", "shifted"])
def test_parallel_eigensolve_at_every_checkpoint(case):
    # forced for every checkpoint (KRY_ERRCTL_BIG=1): the same stops and
    # bounds as the oracle's LAPACK route, as the serial QL gives them
    require_gpu()
    from tests.test_gpu_onepass import env
    if case == "heat3d":
        p = W.small_heat3d(m=10, k=56, steps=100)
        eps = 1e-9
    else:
        p = W.random_symmetric(n=400, ngen=4, o=2, k=40, steps=50, dt=0.05, seed=21, affine=True, center=True)
        diag = p.colidx == np.repeat(np.arange(p.n), np.diff(p.rowptr))
        p.vals = p.vals + 1.2 * diag
        eps = 1e-7
    with env(KRY_ERRCTL_BIG=1):
        _run(p, eps)


def test_stop_past_2048():
    # 1D heat, n = 10^5, a 50-cell start, horizon 8e-6: the bound first
    # drops below 1e-6 at k = 2283 (the oracle's stop)
    require_gpu()
    import math
    n = 100_000
    p = W.heat1d(n=n, k=2600, steps=2, dt=4e-6)      # few steps: the oracle exponentiates each at k = 2283
    p.gens = [W.Generator(W.segments_from_ranges([(n // 3, n // 3 + 50)], 1.0), 1.0, 0.1)]
    p.C = [W.segments_from_ranges([(n // 2 - 10, n // 2 + 10)], 0.05)]
    p.unsafe = np.array([[math.inf, math.inf]])
    errs, ref = _run(p, 1e-6, method=kry.KRY_LANCZOS_PLAIN)
    assert errs[0][0] == ref["runs"][0]["k_stop"] > 2048
