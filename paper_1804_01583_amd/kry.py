"""ctypes binding of libkry.so (include/kry.h).  Argument marshalling only:
every step of the verification path runs in the library's HIP kernels.

The functions keep the C names (kry_plan, kry_plan_create, kry_verify_noalloc, kry_project_expm,
kry_check_box_safety, kry_footprint, kry_plan_workspace, kry_plan_runs, kry_plan_krylov,
kry_plan_block, kry_plan_set_error_target, kry_plan_error, kry_plan_autotune, kry_tune_choice, kry_tune_clear,
kry_plan_destroy, kry_matrix_create,
kry_matrix_bytes, kry_matrix_destroy).  ``Plan`` is a small owner object that keeps the device
tensors a plan borrows alive and destroys the plan when it is dropped.
"""
from __future__ import annotations

import ctypes as ct
import math
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkry.so")

KRY_OK, KRY_EINVAL, KRY_ENOMEM, KRY_EDEVICE, KRY_ENUMERIC, KRY_ENOTSUP = range(6)
KRY_FP64, KRY_FP32_BASIS = 0, 1
KRY_AUTO, KRY_LANCZOS, KRY_ARNOLDI, KRY_BLOCK_ARNOLDI, KRY_LANCZOS_PLAIN = range(5)
KRY_CSR, KRY_STENCIL7 = 0, 1
KRY_BC_DIRICHLET, KRY_BC_INSULATED = 0, 1
ROLE_NAMES = {0: "gen", 1: "center", 2: "affine"}


class KryError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"kry status {status}: {msg}")
        self.status = status


class KrySegs(ct.Structure):
    _fields_ = [("nseg", ct.c_int64), ("lo", ct.c_void_p), ("hi", ct.c_void_p), ("w", ct.c_void_p)]


class KrySystem(ct.Structure):
    _fields_ = [("n", ct.c_int64), ("kind", ct.c_int32), ("symmetric", ct.c_int32),
                ("rowptr", ct.c_void_p), ("colidx", ct.c_void_p), ("vals", ct.c_void_p),
                ("nnz", ct.c_int64), ("nx", ct.c_int64), ("ny", ct.c_int64), ("nz", ct.c_int64),
                ("c0", ct.c_double), ("cx", ct.c_double), ("cy", ct.c_double), ("cz", ct.c_double),
                ("b", ct.c_void_p), ("anorm", ct.c_double), ("b_segs", ct.POINTER(KrySegs)),
                ("prepared", ct.c_void_p), ("stencil_bc", ct.c_int32), ("stencil_exchange", ct.c_double)]


class KryGen(ct.Structure):
    _fields_ = [("seg", KrySegs), ("zc", ct.c_double), ("radius", ct.c_double)]


class KryInterval(ct.Structure):
    _fields_ = [("lo", ct.c_double), ("hi", ct.c_double)]


class KryVerdict(ct.Structure):
    _fields_ = [("first_step", ct.c_int64), ("row", ct.c_int32), ("status", ct.c_int32),
                ("y", ct.c_double), ("lo", ct.c_double), ("hi", ct.c_double)]


def _load():
    # torch ships its own HIP runtime; load it first so libkry.so binds to the
    # same runtime instance (two instances in one process do not share devices)
    import torch  # noqa: F401

    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing; build it with `python -m paper_1804_01583_amd.build`")
    lib = ct.CDLL(LIB_PATH)
    P = ct.c_void_p
    lib.kry_plan_create.argtypes = [ct.POINTER(KrySystem), ct.POINTER(KryGen), ct.c_int32, P,
                                    ct.POINTER(KrySegs), ct.c_int32, ct.c_int32, ct.c_double, ct.c_int64,
                                    ct.c_int32, ct.c_int32, ct.c_int32, P, ct.c_size_t, P, ct.POINTER(P)]
    lib.kry_plan.argtypes = [ct.POINTER(KrySystem), ct.POINTER(KryGen), ct.c_int32, P,
                             ct.POINTER(KrySegs), ct.c_int32, ct.c_int32, ct.c_double, ct.c_int64,
                             ct.c_int32, ct.c_int32, ct.c_int32, P, ct.POINTER(P)]
    lib.kry_verify_noalloc.argtypes = [ct.POINTER(KrySystem), ct.POINTER(KryGen), ct.c_int32, P,
                                       ct.POINTER(KrySegs), ct.c_int32, ct.c_int32, ct.c_double, ct.c_int64,
                                       ct.c_int32, ct.c_int32, ct.c_int32, ct.POINTER(KryInterval), P,
                                       ct.POINTER(KryVerdict), P, P]
    lib.kry_plan_create_transposed.argtypes = [ct.POINTER(KrySystem), ct.POINTER(KryGen), ct.c_int32,
                                               ct.POINTER(KrySegs), ct.POINTER(KrySegs), ct.c_int32, ct.c_int32,
                                               ct.c_double, ct.c_int64, ct.c_int32, ct.c_int32, P, ct.c_size_t, P,
                                               ct.POINTER(P)]
    lib.kry_footprint_transposed.argtypes = [ct.POINTER(KrySystem), ct.c_int32, ct.c_int32, ct.c_int32, ct.c_int32,
                                             ct.c_int64, ct.c_int64, ct.c_int32, ct.c_int32, ct.POINTER(ct.c_size_t)]
    lib.kry_project_expm.argtypes = [P, P]
    lib.kry_check_lp_safety.argtypes = [P, P, P, ct.c_int32, P, P, ct.c_int32, ct.POINTER(ct.c_int64),
                                        ct.POINTER(ct.c_int32), P, P, P]
    lib.kry_check_box_safety.argtypes = [P, ct.POINTER(KryInterval), ct.POINTER(KryVerdict), P]
    lib.kry_check_box_subset.argtypes = [P, P, ct.c_int32, P, ct.c_int32, ct.c_int64, ct.POINTER(KryInterval),
                                         ct.POINTER(KryVerdict), P]
    lib.kry_plan_workspace.argtypes = [ct.POINTER(KrySystem), ct.c_int32, ct.c_int32, ct.c_int32, ct.c_int64,
                                       ct.c_int64, ct.c_int32, ct.c_int32, ct.c_int32, ct.POINTER(ct.c_size_t)]
    lib.kry_footprint.argtypes = [ct.POINTER(KrySystem), ct.c_int32, ct.c_int32, ct.c_int32, ct.c_int32,
                                  ct.c_int32, ct.POINTER(ct.c_size_t)]
    lib.kry_plan_runs.argtypes = [P, ct.POINTER(ct.c_int32), P]
    lib.kry_plan_krylov.argtypes = [P, ct.c_int32, ct.POINTER(ct.c_int32), ct.POINTER(ct.c_double), P,
                                    ct.POINTER(ct.c_double), P]
    lib.kry_plan_block.argtypes = [P, ct.c_int32, ct.POINTER(ct.c_int32), ct.POINTER(ct.c_int32),
                                   ct.POINTER(ct.c_int32), P, P, P]
    lib.kry_plan_set_error_target.argtypes = [P, ct.c_double]
    lib.kry_plan_set_graph.argtypes = [P, ct.c_int32]
    lib.kry_plan_error.argtypes = [P, ct.c_int32, ct.POINTER(ct.c_int32), ct.POINTER(ct.c_double)]
    lib.kry_plan_autotune.argtypes = [P, ct.c_int32, ct.POINTER(ct.c_int32)]
    lib.kry_tune_choice.argtypes = [ct.c_char_p, ct.c_int64, ct.c_int32, ct.POINTER(ct.c_int32),
                                    ct.POINTER(ct.c_int32), ct.POINTER(ct.c_int32), ct.POINTER(ct.c_double)]
    lib.kry_tune_clear.argtypes = []
    lib.kry_tune_clear.restype = None
    lib.kry_matrix_create.argtypes = [ct.POINTER(KrySystem), ct.c_int32, P, ct.POINTER(P)]
    lib.kry_matrix_bytes.argtypes = [P, ct.POINTER(ct.c_size_t)]
    lib.kry_matrix_destroy.argtypes = [P]
    lib.kry_matrix_destroy.restype = None
    lib.kry_plan_destroy.argtypes = [P]
    lib.kry_plan_destroy.restype = None
    lib.kry_last_error.restype = ct.c_char_p
    lib.kry_profile_enable.argtypes = [ct.c_int32]
    lib.kry_profile_read.argtypes = [ct.c_char_p, ct.POINTER(ct.c_int64), ct.POINTER(ct.c_double)]
    lib.kry_profile_names.restype = ct.c_char_p
    for f in ("kry_plan", "kry_plan_create", "kry_verify_noalloc", "kry_plan_create_transposed", "kry_footprint_transposed",
              "kry_project_expm", "kry_check_lp_safety", "kry_check_box_safety", "kry_check_box_subset",
              "kry_footprint", "kry_plan_workspace", "kry_plan_runs", "kry_plan_krylov", "kry_plan_block", "kry_plan_set_error_target",
              "kry_plan_set_graph", "kry_plan_error", "kry_matrix_create", "kry_matrix_bytes", "kry_profile_enable",
              "kry_profile_reset", "kry_profile_read", "kry_plan_autotune", "kry_tune_choice"):
        getattr(lib, f).restype = ct.c_int
    return lib


lib = _load()

EXPORTED = ["kry_plan", "kry_plan_create", "kry_verify_noalloc", "kry_plan_create_transposed", "kry_footprint_transposed",
            "kry_project_expm", "kry_check_lp_safety", "kry_check_box_safety", "kry_check_box_subset",
            "kry_footprint", "kry_plan_workspace", "kry_plan_runs", "kry_plan_krylov", "kry_plan_block", "kry_plan_set_error_target", "kry_plan_set_graph",
            "kry_plan_error", "kry_plan_autotune", "kry_tune_choice", "kry_tune_clear",
            "kry_plan_destroy", "kry_matrix_create", "kry_matrix_bytes", "kry_matrix_destroy", "kry_last_error",
            "kry_profile_enable", "kry_profile_reset", "kry_profile_read", "kry_profile_names"]


def _check(status: int):
    if status != KRY_OK:
        raise KryError(status, lib.kry_last_error().decode(errors="replace"))


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    if hasattr(t, "data_ptr"):
        return t.data_ptr()
    if isinstance(t, np.ndarray):
        return t.ctypes.data
    return int(t)


# ---------------------------------------------------------------------------
# thin wrappers with the C names
# ---------------------------------------------------------------------------

def kry_plan_create(system: KrySystem, gens: Sequence[KryGen], center_ptr, C: Sequence[KrySegs], k: int,
                    dt: float, steps: int, precision=KRY_FP64, method=KRY_AUTO, block_p=0,
                    workspace_ptr=None, workspace_bytes=0, stream_ptr=None) -> int:
    garr = (KryGen * max(len(gens), 1))(*gens)
    carr = (KrySegs * len(C))(*C)
    out = ct.c_void_p()
    _check(lib.kry_plan_create(ct.byref(system), garr, len(gens), center_ptr, carr, len(C), k, dt, steps,
                               precision, method, block_p, workspace_ptr, workspace_bytes, stream_ptr,
                               ct.byref(out)))
    return out.value


def kry_plan(system: KrySystem, gens: Sequence[KryGen], center_ptr, C: Sequence[KrySegs], k: int, dt: float,
             steps: int, precision=KRY_FP64, method=KRY_AUTO, block_p=0, stream_ptr=None) -> int:
    garr = (KryGen * max(len(gens), 1))(*gens)
    carr = (KrySegs * len(C))(*C)
    out = ct.c_void_p()
    _check(lib.kry_plan(ct.byref(system), garr, len(gens), center_ptr, carr, len(C), k, dt, steps, precision,
                        method, block_p, stream_ptr, ct.byref(out)))
    return out.value


def kry_verify_noalloc(system: KrySystem, gens: Sequence[KryGen], center_ptr, C: Sequence[KrySegs], k: int,
                       dt: float, steps: int, unsafe: np.ndarray, basis_out_ptr=None, precision=KRY_FP64,
                       method=KRY_AUTO, block_p=0, stream_ptr=None):
    """Plan, projection and box check in one call on the library's scratch
    array; returns (verdict, z)."""
    garr = (KryGen * max(len(gens), 1))(*gens)
    carr = (KrySegs * len(C))(*C)
    U = (KryInterval * len(unsafe))(*[KryInterval(float(a), float(b)) for a, b in unsafe])
    v = KryVerdict()
    z = np.zeros(max(len(gens), 1))
    _check(lib.kry_verify_noalloc(ct.byref(system), garr, len(gens), center_ptr, carr, len(C), k, dt, steps,
                                  precision, method, block_p, U, basis_out_ptr, ct.byref(v), z.ctypes.data,
                                  stream_ptr))
    return v, z[:len(gens)]


KRY_NOALLOC_SCRATCH_BYTES = 128 << 20


def kry_plan_create_transposed(system_t: KrySystem, gens: Sequence[KryGen], center: Optional[KrySegs],
                               C: Sequence[KrySegs], k: int, dt: float, steps: int, precision=KRY_FP64,
                               method=KRY_AUTO, stream_ptr=None, workspace_ptr=None, workspace_bytes=0) -> int:
    garr = (KryGen * max(len(gens), 1))(*gens)
    carr = (KrySegs * len(C))(*C)
    out = ct.c_void_p()
    cptr = ct.byref(center) if center is not None else None
    _check(lib.kry_plan_create_transposed(ct.byref(system_t), garr, len(gens), cptr, carr, len(C), k, dt, steps,
                                          precision, method, workspace_ptr, workspace_bytes, stream_ptr,
                                          ct.byref(out)))
    return out.value


def kry_footprint_transposed(system_t: KrySystem, ngen: int, has_center: bool, o: int, k: int, steps: int,
                             nseg_total: int, precision=KRY_FP64, method=KRY_AUTO) -> int:
    b = ct.c_size_t()
    _check(lib.kry_footprint_transposed(ct.byref(system_t), ngen, 1 if has_center else 0, o, k, steps, nseg_total,
                                        precision, method, ct.byref(b)))
    return b.value


def kry_project_expm(plan: int, basis_out_ptr=None):
    _check(lib.kry_project_expm(plan, basis_out_ptr))


def kry_check_box_safety(plan: int, unsafe: np.ndarray, ngen: int):
    o = unsafe.shape[0]
    U = (KryInterval * o)(*[KryInterval(float(a), float(b)) for a, b in unsafe])
    v = KryVerdict()
    z = np.zeros(max(ngen, 1))
    _check(lib.kry_check_box_safety(plan, U, ct.byref(v), z.ctypes.data))
    return v, z[:ngen]


def kry_check_box_subset(plan: int, cols, rows, steps: int, unsafe: np.ndarray, ngen: int):
    """The box check over basis columns `cols` and output rows `rows` up to
    `steps`; ngen = generator columns among cols (length of z)."""
    c = np.ascontiguousarray(cols, np.int32)
    r = np.ascontiguousarray(rows, np.int32)
    U = (KryInterval * len(r))(*[KryInterval(float(a), float(b)) for a, b in unsafe])
    v = KryVerdict()
    z = np.zeros(max(ngen, 1))
    _check(lib.kry_check_box_subset(plan, c.ctypes.data, c.size, r.ctypes.data, r.size, steps, U, ct.byref(v),
                                    z.ctypes.data))
    return v, z[:ngen]


def kry_check_lp_safety(plan: int, G, h, U, u, ngen: int, o: int, steps: int, want_flags=False):
    """Per-step LP; returns (first_step, status, z, y, flags or None)."""
    G = np.ascontiguousarray(np.asarray(G, np.float64).reshape(-1, ngen) if ngen else np.zeros((len(h), 0)))
    h = np.ascontiguousarray(h, np.float64)
    U = np.ascontiguousarray(np.asarray(U, np.float64).reshape(-1, o))
    u = np.ascontiguousarray(u, np.float64)
    first = ct.c_int64()
    status = ct.c_int32()
    z = np.zeros(max(ngen, 1))
    y = np.zeros(max(o, 1))
    flags = np.zeros(steps + 1, np.int32) if want_flags else None
    _check(lib.kry_check_lp_safety(plan, G.ctypes.data, h.ctypes.data, h.size, U.ctypes.data, u.ctypes.data, u.size,
                                   ct.byref(first), ct.byref(status), z.ctypes.data, y.ctypes.data,
                                   flags.ctypes.data if want_flags else None))
    return first.value, status.value, z[:ngen], y[:o], flags


def kry_plan_workspace(system: KrySystem, nruns: int, o: int, k: int, steps: int, nseg_total: int,
                       precision=KRY_FP64, method=KRY_AUTO, block_p=0) -> int:
    b = ct.c_size_t()
    _check(lib.kry_plan_workspace(ct.byref(system), nruns, o, k, steps, nseg_total, precision, method, block_p,
                                  ct.byref(b)))
    return b.value


def kry_footprint(system: KrySystem, ngen: int, o: int, k: int, precision=KRY_FP64, block_p=0) -> int:
    b = ct.c_size_t()
    _check(lib.kry_footprint(ct.byref(system), ngen, o, k, precision, block_p, ct.byref(b)))
    return b.value


def kry_plan_runs(plan: int):
    n = ct.c_int32()
    _check(lib.kry_plan_runs(plan, ct.byref(n), None))
    roles = np.zeros(n.value, dtype=np.int32)
    _check(lib.kry_plan_runs(plan, ct.byref(n), roles.ctypes.data))
    return [ROLE_NAMES[int(r)] for r in roles]


def kry_plan_krylov(plan: int, run: int, k: int, o: int):
    keff = ct.c_int32()
    beta0 = ct.c_double()
    hn = ct.c_double()
    H = np.zeros((k + 1) * (k + 1))
    P = np.zeros(o * (k + 1))
    _check(lib.kry_plan_krylov(plan, run, ct.byref(keff), ct.byref(beta0), H.ctypes.data, ct.byref(hn),
                               P.ctypes.data))
    m = keff.value
    return {"k_eff": m, "beta0": beta0.value, "H": H[:m * m].reshape(m, m).copy(),
            "h_next": hn.value, "P": P[:o * m].reshape(o, m).copy()}


def kry_matrix_create(system: KrySystem, precision=KRY_FP64, stream_ptr=None) -> int:
    out = ct.c_void_p()
    _check(lib.kry_matrix_create(ct.byref(system), precision, stream_ptr, ct.byref(out)))
    return out.value


def kry_matrix_bytes(mat: int) -> int:
    b = ct.c_size_t()
    _check(lib.kry_matrix_bytes(mat, ct.byref(b)))
    return b.value


def kry_matrix_destroy(mat: int):
    lib.kry_matrix_destroy(mat)


def kry_plan_set_error_target(plan: int, eps: float):
    _check(lib.kry_plan_set_error_target(plan, eps))


def kry_plan_set_graph(plan: int, on: bool):
    _check(lib.kry_plan_set_graph(plan, 1 if on else 0))


def kry_plan_autotune(plan: int, reps: int = 5) -> int:
    """kry_plan_autotune: kernels tuned for this plan's shape."""
    tuned = ct.c_int32()
    _check(lib.kry_plan_autotune(plan, reps, ct.byref(tuned)))
    return tuned.value


def kry_tune_choice(kernel: str, n: int, runs: int):
    """The stored choice (a, b, microseconds) or None."""
    found, a, b, us = ct.c_int32(), ct.c_int32(), ct.c_int32(), ct.c_double()
    _check(lib.kry_tune_choice(kernel.encode(), n, runs, ct.byref(found), ct.byref(a), ct.byref(b), ct.byref(us)))
    return (a.value, b.value, us.value) if found.value else None


def kry_tune_clear():
    lib.kry_tune_clear()


def kry_plan_error(plan: int, run: int):
    """(k_used, bound) of one run."""
    k = ct.c_int32()
    b = ct.c_double()
    _check(lib.kry_plan_error(plan, run, ct.byref(k), ct.byref(b)))
    return k.value, b.value


def kry_plan_block(plan: int, block: int, o: int):
    """Block run `block` of a block Arnoldi plan: k_eff, p, H, R0, P (or the
    number of block runs when block < 0)."""
    nb, keff, pp = ct.c_int32(), ct.c_int32(), ct.c_int32()
    _check(lib.kry_plan_block(plan, -1, ct.byref(nb), None, None, None, None, None))
    if block < 0:
        return nb.value
    _check(lib.kry_plan_block(plan, block, None, ct.byref(keff), ct.byref(pp), None, None, None))
    m = keff.value * pp.value
    H = np.zeros(max(m * m, 1))
    R0 = np.zeros(max(pp.value * pp.value, 1))
    Pm = np.zeros(max(o * m, 1))
    _check(lib.kry_plan_block(plan, block, None, None, None, H.ctypes.data, R0.ctypes.data, Pm.ctypes.data))
    return {"k_eff": keff.value, "p": pp.value, "H": H[:m * m].reshape(m, m).copy(),
            "R0": R0[:pp.value ** 2].reshape(pp.value, pp.value).copy(), "P": Pm[:o * m].reshape(o, m).copy()}


def kry_plan_destroy(plan: int):
    lib.kry_plan_destroy(plan)


def profile_enable(on: bool = True):
    _check(lib.kry_profile_enable(1 if on else 0))


def profile_reset():
    _check(lib.kry_profile_reset())


def profile_read(name: str):
    n = ct.c_int64()
    ms = ct.c_double()
    _check(lib.kry_profile_read(name.encode(), ct.byref(n), ct.byref(ms)))
    return n.value, ms.value


def profile_names():
    return lib.kry_profile_names().decode().split(",")


# ---------------------------------------------------------------------------
# owner object
# ---------------------------------------------------------------------------

def _segs(seg, keep) -> KrySegs:
    lo = np.ascontiguousarray(seg.lo, dtype=np.int64)
    hi = np.ascontiguousarray(seg.hi, dtype=np.int64)
    w = np.ascontiguousarray(seg.w, dtype=np.float64)
    keep += [lo, hi, w]
    return KrySegs(lo.size, lo.ctypes.data, hi.ctypes.data, w.ctypes.data)


class _Runs:
    """Index ranges [lo, hi) with one value each (the layout of kry_segs)."""

    def __init__(self, lo, hi, w):
        self.lo, self.hi, self.w = lo, hi, w


def _runs_of(v) -> _Runs:
    """A dense host vector as maximal runs of equal nonzero entries (a change
    of format for the library's segment sets)."""
    v = np.asarray(v, np.float64)
    nz = v != 0.0
    # a run starts where an entry is nonzero and differs from its left neighbour
    # (or that neighbour is zero); it ends before the next start or zero
    start = nz & np.concatenate(([True], (v[1:] != v[:-1]) | ~nz[:-1]))
    lo = np.flatnonzero(start)
    stop = np.flatnonzero(nz & np.concatenate(((v[1:] != v[:-1]) | ~nz[1:], [True]))) + 1
    return _Runs(lo.astype(np.int64), stop.astype(np.int64), v[lo])


class DeviceSystem:
    """The system matrix, forcing and optional center of a problem in device
    memory (torch tensors), uploaded once and reusable by many plans.
    ``problem`` is any object with the attributes of workloads.Problem."""

    def __init__(self, problem, device="cuda"):
        import torch
        self.problem = problem
        self.device = device
        self.tensors = []
        s = KrySystem()
        s.n = problem.n
        s.symmetric = 1 if problem.symmetric else 0
        if problem.kind == "csr":
            s.kind = KRY_CSR
            self.rowptr = torch.as_tensor(np.asarray(problem.rowptr, np.int64), device=device)
            self.colidx = torch.as_tensor(np.asarray(problem.colidx, np.int32), device=device)
            self.vals = torch.as_tensor(np.asarray(problem.vals, np.float64), device=device)
            s.rowptr, s.colidx, s.vals = _ptr(self.rowptr), _ptr(self.colidx), _ptr(self.vals)
            s.nnz = int(self.colidx.numel())
        else:
            s.kind = KRY_STENCIL7
            s.nx, s.ny, s.nz = problem.grid
            s.c0, s.cx, s.cy, s.cz = problem.coef
            s.stencil_bc = KRY_BC_INSULATED if getattr(problem, "bc", "dirichlet") == "insulated" else KRY_BC_DIRICHLET
            s.stencil_exchange = float(getattr(problem, "exchange", 0.0))
        self.b = None
        self._keep = []
        if problem.b is not None:
            self.b = torch.as_tensor(np.asarray(problem.b, np.float64), device=device)
            s.b = _ptr(self.b)
        elif getattr(problem, "b_seg", None) is not None:
            self._bseg = _segs(problem.b_seg, self._keep)
            s.b_segs = ct.pointer(self._bseg)
        self.center = None
        if problem.center is not None:
            self.center = torch.as_tensor(np.asarray(problem.center, np.float64), device=device)
        s.anorm = 0.0
        s.prepared = None
        self.sys = s
        self.prepared = {}
        self._marshalled = None      # the problem's generators and outputs as kry_gen / kry_segs
        self._footprints = {}        # workspace bytes per plan shape
        self._runs = {}              # index runs of the dense center / forcing (transposed plans)

    def prepare(self, precision=KRY_FP64, stream=None):
        """kry_matrix_create for this CSR system and precision, once: plans of
        that precision then share its sliced-ELL copy and norm."""
        if precision not in self.prepared:
            sp = None if stream is None else stream.cuda_stream
            self.prepared[precision] = kry_matrix_create(self.sys, precision, sp)
        return self.prepared[precision]

    def runs_of(self, name) -> "_Runs":
        """The problem's dense vector ``name`` (center or b) as index runs,
        converted once: like the uploaded vectors, it is read when the
        system is made."""
        r = self._runs.get(name)
        if r is None:
            r = self._runs[name] = _runs_of(getattr(self.problem, name))
        return r

    def system_for(self, precision) -> KrySystem:
        """The kry_system a plan of `precision` gets (with its prepared matrix)."""
        s = KrySystem.from_buffer_copy(self.sys)
        s.prepared = self.prepared.get(precision)
        return s

    def close(self):
        for h in self.prepared.values():
            kry_matrix_destroy(h)
        self.prepared = {}

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 - interpreter shutdown
            pass


class Plan:
    """kry_plan_create + owned references.  ``workspace``: 'torch' takes the
    workspace from torch's caching allocator, 'library' lets the plan
    allocate its own."""

    def __init__(self, dsys: DeviceSystem, k=None, dt=None, steps=None, precision=KRY_FP64,
                 method=KRY_AUTO, block_p=0, stream=None, workspace="torch", gens=None, C=None):
        import torch
        p = dsys.problem
        self.dsys = dsys
        self._sys = dsys.system_for(precision)
        self.k = p.k if k is None else k
        self.dt = p.dt if dt is None else dt
        self.steps = p.steps if steps is None else steps
        own = gens is None and C is None
        gens = p.gens if gens is None else gens
        C = p.C if C is None else C
        self.ngen = len(gens)
        self.o = len(C)
        # the problem's own generators and outputs are marshalled once per
        # device system (plans of one system reuse them)
        if own and dsys._marshalled is not None:
            self._gens, self._C, self._keep = dsys._marshalled
        else:
            keep = []
            self._gens = [KryGen(_segs(g.seg, keep), float(g.zc), float(g.radius)) for g in gens]
            self._C = [_segs(c, keep) for c in C]
            self._keep = keep
            if own:
                dsys._marshalled = (self._gens, self._C, keep)
        has_forcing = dsys.b is not None or getattr(p, "b_seg", None) is not None
        nruns = self.ngen + (dsys.center is not None) + has_forcing
        self.stream = torch.cuda.current_stream(dsys.device) if stream is None else stream
        ws_ptr, ws_bytes = None, 0
        self.workspace = None
        if workspace == "torch":
            nseg = sum(g.seg.nseg for g in self._gens) + sum(c.nseg for c in self._C)
            if getattr(p, "b_seg", None) is not None and dsys.b is None:
                nseg += p.b_seg.nseg
            key = (own, precision, method, block_p, self.k, self.steps, nseg, self.o, nruns, self._sys.prepared)
            ws_bytes = dsys._footprints.get(key) if own else None
            if ws_bytes is None:
                ws_bytes = kry_plan_workspace(self._sys, max(nruns, 1), self.o, self.k, self.steps, nseg, precision,
                                         method, block_p)
                if own:
                    dsys._footprints[key] = ws_bytes
            self.workspace = torch.empty(ws_bytes, dtype=torch.uint8, device=dsys.device)
            ws_ptr = self.workspace.data_ptr()
        self.handle = None
        self.handle = kry_plan_create(self._sys, self._gens, _ptr(dsys.center), self._C, self.k, self.dt,
                                      self.steps, precision, method, block_p, ws_ptr, ws_bytes,
                                      self.stream.cuda_stream)
        self.roles = kry_plan_runs(self.handle)

    @property
    def nruns(self):
        return len(self.roles)

    def project_expm(self, out=None):
        """Runs the Krylov processes and fills the basis; ``out`` may be a
        torch tensor (device or host) of shape (steps+1, o, nruns)."""
        kry_project_expm(self.handle, _ptr(out))
        return out

    def basis(self):
        import torch
        out = torch.empty((self.steps + 1, self.o, self.nruns), dtype=torch.float64)
        kry_project_expm(self.handle, out.data_ptr())
        return out.numpy()

    def check(self, unsafe):
        v, z = kry_check_box_safety(self.handle, np.asarray(unsafe, np.float64), self.ngen)
        return {"first_step": int(v.first_step), "row": int(v.row), "status": int(v.status), "y": v.y,
                "lo": v.lo, "hi": v.hi, "z": z}

    def check_lp(self, G, h, U, u, flags=False):
        """The per-step LP (kry_check_lp_safety): initial set = the generator
        box and G z <= h, unsafe set U y <= u.  Needs project_expm first."""
        first, status, z, y, fl = kry_check_lp_safety(self.handle, G, h, U, u, self.ngen, self.o, self.steps, flags)
        return {"first_step": first, "status": status, "z": z, "y": y, "flags": fl}

    def krylov(self, run: int):
        return kry_plan_krylov(self.handle, run, self.k, self.o)

    def set_graph(self, on: bool = True):
        """Graph mode (kry_plan_set_graph): project_expm records its launches
        once and replays them."""
        kry_plan_set_graph(self.handle, on)

    def set_error_target(self, eps: float):
        """Error-controlled Krylov dimension (see kry_plan_set_error_target)."""
        kry_plan_set_error_target(self.handle, eps)

    def autotune(self, reps: int = 5) -> int:
        """kry_plan_autotune: kernels tuned (choices that change no value)."""
        return kry_plan_autotune(self.handle, reps)

    def error(self, run: int):
        """(k_used, bound) of a run after project_expm."""
        return kry_plan_error(self.handle, run)

    def blocks(self):
        """Block Arnoldi plans: one dict per block run (see kry_plan_block)."""
        return [kry_plan_block(self.handle, b, self.o) for b in range(kry_plan_block(self.handle, -1, self.o))]

    def close(self):
        if self.handle:
            kry_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class TransposedPlan(Plan):
    """kry_plan_create_transposed: the basis by one run of A^T per output row
    (Section 4.1).  ``dsys_t`` holds the transposed matrix (for a symmetric
    system, the system itself); generators, center, forcing and outputs are
    those of ``dsys_t.problem`` unless given.  A dense forcing or center is
    handed to the library as index ranges.  ``workspace``: 'torch' takes the
    workspace (kry_footprint_transposed bytes) from torch's caching
    allocator, 'library' lets the plan allocate its own."""

    def __init__(self, dsys_t: DeviceSystem, k=None, dt=None, steps=None, precision=KRY_FP64, method=KRY_AUTO,
                 stream=None, gens=None, C=None, workspace="torch"):
        import torch
        p = dsys_t.problem
        self.dsys = dsys_t
        self._sys = dsys_t.system_for(precision)
        self.k = p.k if k is None else k
        self.dt = p.dt if dt is None else dt
        self.steps = p.steps if steps is None else steps
        gens = p.gens if gens is None else gens
        C = p.C if C is None else C
        self.ngen = len(gens)
        self.o = len(C)
        keep = []
        self._gens = [KryGen(_segs(g.seg, keep), float(g.zc), float(g.radius)) for g in gens]
        self._C = [_segs(c, keep) for c in C]
        self._center = _segs(dsys_t.runs_of("center"), keep) if p.center is not None else None
        if p.b is not None:
            self._bseg = _segs(dsys_t.runs_of("b"), keep)
            self._sys.b = None
            self._sys.b_segs = ct.pointer(self._bseg)
        self._keep = keep
        self.workspace = None
        self.stream = torch.cuda.current_stream(dsys_t.device) if stream is None else stream
        ws_ptr, ws_bytes = None, 0
        if workspace not in ("torch", "library"):
            raise ValueError(f"workspace must be 'torch' or 'library', not {workspace!r}")
        if workspace == "torch":
            nseg = sum(g.seg.nseg for g in self._gens) + sum(c.nseg for c in self._C)
            nseg += (self._center.nseg if self._center is not None else 0)
            if self._sys.b_segs:
                nseg += self._sys.b_segs.contents.nseg
            ws_bytes = kry_footprint_transposed(self._sys, self.ngen, self._center is not None, self.o, self.k,
                                                self.steps, nseg, precision, method)
            self.workspace = torch.empty(ws_bytes, dtype=torch.uint8, device=dsys_t.device)
            ws_ptr = self.workspace.data_ptr()
        self.handle = None
        self.handle = kry_plan_create_transposed(self._sys, self._gens, self._center, self._C, self.k, self.dt,
                                                 self.steps, precision, method, self.stream.cuda_stream, ws_ptr,
                                                 ws_bytes)
        self.runs = kry_plan_runs(self.handle)
        self.ncols = self.ngen + (p.center is not None) + (p.b is not None or getattr(p, "b_seg", None) is not None)
        self.roles = ["gen"] * self.ngen + (["center"] if p.center is not None else []) + \
            (["affine"] if self.ncols > self.ngen + (p.center is not None) else [])

    def krylov(self, run: int):
        """Transposed run ``run`` (output row): P has one row per basis column."""
        return kry_plan_krylov(self.handle, run, self.k, self.ncols)
