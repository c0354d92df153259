"""Throughput of one verification of the 3D heat system (100^3 grid, n = 10^6,
7-point stencil stored as CSR, affine forcing, Lanczos k = 40, dt = 0.02,
2000 steps, FP64) on one GPU.

A step is the whole path on one batch of input already resident in HBM:
plan (run split, start vectors), the Krylov process of every run, the
per-step exponentials and basis assembly, and the box safety check with its
verdict copied back to the host.  value = verified time-steps per second,
(steps + 1) * runs / seconds per step.

Prints one JSON line.  Options:
  --gpus N        only N = 1 is supported (one process, one GPU)
  --steps K       timed steps (default 20)
  --warmup W      untimed steps first (default 3)
  --no-cpu-baseline   skip timing the CPU oracle
  --m M           grid edge (default 100)
  --calib-copy    run a plain device copy of known size (for counter calibration) and exit
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def calib_copy(torch):
    nbytes = 1 << 30
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    log(f"calib-copy: 5 copies of {nbytes} bytes (read {nbytes}, write {nbytes} per copy)")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--m", type=int, default=None, help="grid edge (default 100; 1000 for heat3d_stencil)")
    ap.add_argument("--workload", default="heat3d_csr",
                    choices=["heat3d_csr", "heat3d_stencil", "heat1d", "conv_diff3d"],
                    help="heat3d_csr is the benchmark line; the others are measured the same way")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calib-copy", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: --gpus {args.gpus} is not supported "
              "(independent runs and queries shard without communication; see DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    if args.calib_copy:
        calib_copy(torch)
        return
    import workloads as W
    from paper_1804_01583_amd import kry

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    log("building inputs")
    if args.workload == "heat3d_csr":
        p = W.heat3d_csr(m=args.m or 100)
    elif args.workload == "heat3d_stencil":
        p = W.heat3d_stencil(m=args.m or 1000)
    elif args.workload == "heat1d":
        p = W.heat1d()
    else:
        p = W.conv_diff3d(*(((args.m,) * 3) if args.m else (200, 200, 250)), ngen=2, o=5, k=30)
    dsys = kry.DeviceSystem(p, device="cuda")
    stream = torch.cuda.current_stream()

    def step():
        plan = kry.Plan(dsys, stream=stream)
        plan.project_expm(None)
        v = plan.check(p.unsafe)
        nr = plan.nruns
        plan.close()
        return v, nr

    log(f"warmup {args.warmup}")
    for _ in range(args.warmup):
        verdict, nruns = step()
    torch.cuda.synchronize()
    # timed region 1: the whole job, no instrumentation -> value
    log(f"timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        verdict, nruns = step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    # timed region 2: the same steps with every kernel launch bracketed by HIP
    # events on the plan's stream -> per-kernel durations for the roofline
    log(f"timing {args.steps} steps with per-kernel events")
    kry.profile_enable(True)
    kry.profile_reset()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        verdict, nruns = step()
    torch.cuda.synchronize()
    elapsed_ev = time.perf_counter() - t1
    kry.profile_enable(False)
    kern = {}
    for name in kry.profile_names():
        cnt, ms = kry.profile_read(name)
        if cnt:
            kern[name] = {"launches": cnt, "avg_us": 1000.0 * ms / cnt, "total_ms_per_step": ms / args.steps}
    ms_per_step = 1000.0 * elapsed / args.steps
    verified = (p.steps + 1) * nruns
    value = verified / (elapsed / args.steps)

    # algorithmic bytes per launch (all runs of the plan advanced by one launch)
    n, nnz = p.n, p.nnz
    P = nruns
    dom_name = "spmv_csr" if p.kind == "csr" else "spmv_stencil"
    if p.kind == "csr":
        spmv_bytes = 12 * nnz + 8 * (n + 1) + 3 * 8 * n * P     # A (val+col), rowptr, read v_j, v_{j-1}, write w
    else:
        spmv_bytes = 3 * 8 * n * P                              # read v_j, v_{j-1}, write w (matrix-free)
    sweep_bytes = 3 * 8 * n * P                                 # read v_j, w; write w
    for name, b in ((dom_name, spmv_bytes), ("sweep", sweep_bytes)):
        if name in kern:
            kern[name]["bytes"] = b
            kern[name]["GBps"] = b / (kern[name]["avg_us"] * 1e-6) / 1e9
    dom = kern.get(dom_name, {})
    achieved = dom.get("GBps", 0.0)
    traffic = None
    if args.workload == "heat3d_csr" and (args.m or 100) == 100:
        traffic = counter_traffic(os.path.join(ROOT, "profiles", "spmv_csr_heat3d_m100_pmc.md"))
    # Lanczos iteration = spmv + sweep: bytes and time of both kernels
    step_bytes = spmv_bytes + sweep_bytes
    step_us = dom.get("avg_us", 0.0) + kern.get("sweep", {}).get("avg_us", 0.0)

    cpu = None
    if not args.no_cpu_baseline and p.n <= 2_000_000:
        log("timing the CPU oracle on the same workload (one whole verification)")
        cpu = cpu_baseline(p)

    out = {
        "metric": "Krylov step HBM GB/s (% peak); verified time-steps/s vs plain FP64; p99 query latency",
        "value": value,
        "unit": "verified time-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": describe(p, nruns), "n": n, "nnz": nnz, "k": p.k, "time_steps": p.steps,
                   "runs": nruns, "precision": "fp64", "method": "lanczos" if p.symmetric else "arnoldi"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS, "traffic": traffic, "kernel": dom_name,
                     "bytes_per_launch": spmv_bytes},
        "ms_per_step_with_kernel_events": 1000.0 * elapsed_ev / args.steps,
        "krylov_iteration": {"bytes": step_bytes, "us": step_us,
                             "GBps": step_bytes / (step_us * 1e-6) / 1e9 if step_us else None},
        "kernels": kern,
        "verdict": {"first_step": verdict["first_step"], "row": verdict["row"]},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


def describe(p, nruns):
    if p.name == "heat3d_csr":
        m = p.meta["m"]
        return (f"3D heat {m}^3 CSR (n={p.n}, nnz={p.nnz}) + affine forcing, Lanczos k={p.k}, dt={p.dt}, "
                f"{p.steps} steps, o={p.o}, runs={nruns}, FP64")
    if p.name == "heat3d_stencil":
        m = p.meta["m"]
        return (f"3D heat {m}^3 matrix-free 7-point (n={p.n}) + affine forcing, Lanczos k={p.k}, dt={p.dt}, "
                f"{p.steps} steps, o={p.o}, runs={nruns}, FP64")
    return f"{p.name} n={p.n} nnz={p.nnz} k={p.k} dt={p.dt} steps={p.steps} o={p.o} runs={nruns} FP64"


def counter_traffic(path):
    """HBM bytes per launch of the dominant kernel from the committed
    rocprofv3 counter summary: FETCH_SIZE and WRITE_SIZE (KiB per dispatch),
    each scaled by what the same counter reads for a plain 1 GiB device copy.
    None when the summary is missing or was taken on a different kernel
    source than the one built now."""
    import hashlib
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and line.strip().startswith("- "):
            key, _, val = line.strip()[2:].partition(":")
            vals[key.strip()] = val.strip().strip("`")
    try:
        src = os.path.join(ROOT, "paper_1804_01583_amd", "csrc", "kry_lanczos.hip")
        if hashlib.sha256(open(src, "rb").read()).hexdigest() != vals["kernel_source_sha256"]:
            return None
        rd = float(vals["fetch_kib_per_launch"]) * 1024 * float(vals["calib_read_factor"])
        wr = float(vals["write_kib_per_launch"]) * 1024 * float(vals["calib_write_factor"])
        return rd + wr
    except (KeyError, ValueError):
        return None


def cpu_baseline(p):
    """The oracle as it stands, on this host's CPU, one thread, over one whole
    verification of the same workload."""
    try:
        from threadpoolctl import threadpool_limits
    except Exception:   # pragma: no cover
        threadpool_limits = None
    import oracle
    t0 = time.perf_counter()
    if threadpool_limits is not None:
        with threadpool_limits(limits=1):
            res = oracle.verify(p)
    else:
        res = oracle.verify(p)
    dt = time.perf_counter() - t0
    nruns = res["basis"].shape[2]
    return {"value": (p.steps + 1) * nruns / dt, "unit": "verified time-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"one whole verification of the same workload ({dt:.1f} s, {nruns} runs, "
                      f"{p.steps + 1} time points)"}


if __name__ == "__main__":
    main()
