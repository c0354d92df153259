"""Throughput of one verification of the matrix-free 3D heat system (1000^3
grid, n = 10^9, 7-point stencil applied on the fly, affine forcing, Lanczos
k = 20, dt = 0.01, 500 steps, FP64) on one GPU: the largest configuration
that fits one MI355X.

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
  --m M           grid edge (default 1000 for heat3d_stencil, 100 otherwise)
  --workload W    heat3d_stencil (1000^3 matrix-free, the benchmark line),
                  heat3d_csr (100^3 CSR; its working set fits the 256 MB MALL),
                  heat1d, conv_diff3d, heat3d_paper, heat3d_many_inputs (eight
                  initial-space columns, one output), heat3d_many_gens (--ngen
                  box generators, default 256, plus center and forcing; one output)
  --no-fp32-side  heat3d_stencil: skip the FP32-basis side measurement (ratio to
                  FP64 and per-output error against the FP64 basis)
  --route R       forward (one run per column of E) or transposed (one run of A^T
                  per output row, Section 4.1); default transposed for
                  heat3d_many_inputs and heat3d_many_gens, forward otherwise
  --graph         one plan whose projection is recorded as a HIP graph and replayed
                  each step (plan creation outside the timed region; a separate
                  measurement, not the default line)
  --check C       box (the range check of each output row's interval, default) or
                  lp (the per-step LP of Section 2.1: the generator box cut by
                  sum_j (z_j - zc_j) / r_j <= d / 2, unsafe when every output row
                  is in its interval at once)
  --precision P   fp64 (default) or fp32 (FP32-basis mode; the FP64 path is then
                  timed too, for the ratio to plain FP64)
  --method M      auto (Lanczos / Arnoldi by symmetry) or block (block Arnoldi,
                  the default for conv_diff3d: 16 generators as one p = 16 block)
  --workload serve   the serving stream instead: --rates R1,R2,.. (queries/s),
                  --seconds T of arrivals per rate (at most 2000 queries), --slots S,
                  --serve-batch on|off|both (same-step queries of one system in one plan);
                  reports p50/p99 arrival-to-verdict latency per rate
  --autotune      before timing, tune the launch choices that change no value
                  (block mat-vec shape, marching store kind) on one plan
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
# the last-level cache (MALL, Infinity Cache) of MI355X: a kernel whose bytes
# per launch fit in it is not measured against HBM alone
MALL_BYTES = 256 * 2**20
# per workload: the committed rocprofv3 counter summary of the dominant
# kernel and the sources that kernel is built from
COUNTER_PROFILES = {
    "heat3d_stencil": ("lz1_march_heat3d_m1000_pmc.md", ("kry_lz1.hip", "kry_device.h")),
    "heat3d_csr": ("spmv_sell_heat3d_m100_pmc.md", ("kry_sell.hip", "kry_device.h")),
}


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
    ap.add_argument("--k", type=int, default=None, help="Krylov dimension (matrix-free paper heat only)")
    ap.add_argument("--no-kernel-events", action="store_true",
                    help="skip the second timed pass with per-kernel events (long runs)")
    ap.add_argument("--ngen", type=int, default=0, help="heat3d_many_gens: generators (default 256)")
    ap.add_argument("--workload", default="heat3d_stencil",
                    choices=["heat3d_csr", "heat3d_stencil", "heat1d", "conv_diff3d", "heat3d_paper", "heat3d_many_gens",
                             "heat3d_many_inputs", "serve"],
                    help="heat3d_stencil is the benchmark line; the others are measured the same way")
    ap.add_argument("--no-fp32-side", action="store_true")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--route", default=None, choices=["forward", "transposed"])
    ap.add_argument("--check", default="box", choices=["box", "lp"])
    ap.add_argument("--graph", action="store_true")
    ap.add_argument("--method", default=None, choices=["auto", "block", "plain"])
    ap.add_argument("--rates", default="5,10,20,50,100,200")
    ap.add_argument("--seconds", type=float, default=10.0)
    ap.add_argument("--slots", type=int, default=8)
    ap.add_argument("--serve-batch", choices=["on", "off", "both"], default="on")
    ap.add_argument("--error-target", type=float, default=0.0,
                    help="Lanczos workloads: choose each run's Krylov dimension by the Lemma 1 bound (k is the cap)")
    ap.add_argument("--no-prepared", action="store_true",
                    help="CSR: every plan builds its own sliced-ELL copy and norm instead of sharing one")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--autotune", action="store_true",
                    help="time the order-neutral launch choices on one plan first (kry_plan_autotune)")
    ap.add_argument("--calib-copy", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: --gpus {args.gpus} is not supported "
              "(independent runs and queries shard without communication)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    if args.calib_copy:
        calib_copy(torch)
        return
    import workloads as W
    from paper_1804_01583_amd import kry

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.workload == "serve":
        serve_bench(args)
        return
    log("building inputs")
    if args.workload == "heat3d_csr":
        p = W.heat3d_csr(m=args.m or 100)
    elif args.workload == "heat3d_stencil":
        p = W.heat3d_stencil(m=args.m or 1000)
    elif args.workload == "heat1d":
        p = W.heat1d()
    elif args.workload == "heat3d_paper":
        # the paper's heat benchmark (Section 5.3): up to 160^3 as CSR with its
        # error-controlled k (target 1e-6); larger grids matrix-free, at the
        # paper's k = 5932, or with --error-target by the bound up to k = 8192
        m = args.m or 100
        if m <= 160:
            p = W.heat3d_paper(m=m)
            if not args.error_target:
                args.error_target = 1e-6
        else:
            p = W.heat3d_paper_stencil(m=m, k=args.k or (8192 if args.error_target else 5932))
    elif args.workload == "heat3d_many_inputs":
        p = W.heat3d_many_inputs(m=args.m or 100)
    elif args.workload == "heat3d_many_gens":
        p = W.heat3d_many_gens(m=args.m or 100, ngen=args.ngen or 256)
    else:
        p = W.conv_diff3d(*(((args.m,) * 3) if args.m else (200, 200, 250)), ngen=16, o=5, k=30)
    transposed = (args.route or ("transposed" if args.workload in ("heat3d_many_inputs", "heat3d_many_gens")
                                 else "forward")) == "transposed"
    method_name = args.method or {"conv_diff3d": "block", "heat3d_paper": "plain"}.get(args.workload, "auto")
    method = {"block": kry.KRY_BLOCK_ARNOLDI, "plain": kry.KRY_LANCZOS_PLAIN}.get(method_name, kry.KRY_AUTO)
    dsys = kry.DeviceSystem(p, device="cuda")
    f32 = args.precision == "fp32"
    prepared = p.kind == "csr" and not args.no_prepared
    if prepared:
        # the system's sliced-ELL copy and norm, built once like the upload of A
        for prec in ((kry.KRY_FP32_BASIS, kry.KRY_FP64) if f32 else (kry.KRY_FP64,)):
            dsys.prepare(prec)
        torch.cuda.synchronize()
    tuned = None
    if args.autotune and not transposed:
        # one plan's kernels timed before the timed region; the process keeps
        # the choices (every choice gives the same basis bit for bit)
        tp = kry.Plan(dsys, precision=kry.KRY_FP32_BASIS if f32 else kry.KRY_FP64, method=method)
        tuned = {"kernels_tuned": tp.autotune(reps=3)}
        tp.close()
        for kname, runs in (("bspmm", 16), ("bspmm32", 16), ("lz1_march", 2)):
            c = kry.kry_tune_choice(kname, p.n, runs)
            if c is not None:
                tuned[kname] = {"a": c[0], "b": c[1], "us": c[2]}
        log(f"autotune: {tuned}")
    m = measure(torch, kry, p, dsys, kry.KRY_FP32_BASIS if f32 else kry.KRY_FP64, args.steps, args.warmup, method,
                args.error_target, not args.no_kernel_events and not args.graph, transposed, args.check, args.graph)
    fp64_ref = None
    if f32:
        torch.cuda.empty_cache()
        log("plain FP64 on the same workload, for the ratio")
        m64 = measure(torch, kry, p, dsys, kry.KRY_FP64, args.steps, args.warmup, method, args.error_target,
                      True, transposed)
        fp64_ref = {"value": m64["value"], "ms_per_step": m64["ms_per_step"],
                    "ratio_fp32_over_fp64": m["value"] / m64["value"]}
    kern, nruns, verdict = m["kern"], m["nruns"], m["verdict"]
    n, nnz = p.n, p.nnz
    dom_name = m["dom_name"]
    dom = kern.get(dom_name, {})
    achieved = dom.get("GBps", 0.0)
    traffic = None
    default_m = {"heat3d_stencil": 1000}.get(args.workload, 100)
    if args.workload in COUNTER_PROFILES and (args.m or default_m) == default_m and not f32:
        fname, sources = COUNTER_PROFILES[args.workload]
        traffic = counter_traffic(os.path.join(ROOT, "profiles", fname), sources)
    fp32_side = None
    if args.workload == "heat3d_stencil" and not f32 and not args.no_fp32_side and not args.graph:
        torch.cuda.empty_cache()
        log("FP32-basis side measurement on the same workload")
        fp32_side = fp32_side_measure(torch, kry, p, dsys, m, method)

    cpu = None
    if not args.no_cpu_baseline:
        if args.workload == "heat3d_stencil":
            log("timing the CPU oracle on the locality sub-grids (the same result)")
            cpu = cpu_baseline_subgrids(p)
        elif p.n <= 2_000_000:
            log("timing the CPU oracle on the same workload (one whole verification)")
            cpu = cpu_baseline(p, transposed, args.check)

    out = {
        "metric": "Krylov step HBM GB/s (% peak); verified time-steps/s vs plain FP64; p99 query latency",
        "value": m["value"],
        "unit": "verified time-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": m["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if not f32 else "f32-storage/f64-arith",
        "data": "synthetic",
        "config": {"workload": describe(p, nruns, args.precision, method_name), "n": n, "nnz": nnz, "k": p.k,
                   "time_steps": p.steps, "basis_columns": nruns, "krylov_runs": m["krylov_runs"],
                   "route": "transposed" if transposed else "forward", "precision": args.precision,
                   "check": args.check,
                   "graph": ("one plan made before the timed region, its projection replayed as a HIP graph"
                             if args.graph else None),
                   "method": {"block": "block_arnoldi", "plain": "lanczos_plain"}.get(
                       method_name, "lanczos" if p.symmetric else "arnoldi"),
                   "error_target": args.error_target or None,
                   "matrix": ("prepared once (sliced-ELL copy and norm shared by every verification)" if prepared
                              else ("built by every plan" if p.kind == "csr" else "matrix-free stencil"))},
        "roofline": {"bound": "hbm" if (dom.get("bytes") or 0) > MALL_BYTES else "mall",
                     "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS, "traffic": traffic, "kernel": dom_name,
                     "bytes_per_launch": dom.get("bytes"),
                     "note": (None if (dom.get("bytes") or 0) > MALL_BYTES else
                              "bytes per launch fit the 256 MB MALL: an effective rate, not HBM alone")},
        "ms_per_step_with_kernel_events": m["ms_per_step_ev"],
        "kernels": kern,
        "fp64_reference": fp64_ref,
        "fp32_basis_side": fp32_side,
        "error_control": m.get("error_control"),
        "autotune": tuned,
        "verdict": {"first_step": verdict["first_step"], "row": verdict["row"]},
        "cpu_baseline": cpu,
    }
    if args.graph or not dom.get("bytes"):
        # per-kernel events and graph replay exclude each other; without
        # events (--no-kernel-events) there is no launch duration either
        out["roofline"] = None
    print(json.dumps(out))


def serve_bench(args):
    """The serving stream at each rate: count = min(2000, rate * seconds)
    queries with seeded Poisson arrivals, played in real time against the
    resident systems; latency = verdict time - arrival time."""
    import workloads as W
    from paper_1804_01583_amd.serve import Catalog, Server, summarize
    rates = [float(r) for r in args.rates.split(",") if r]
    cat = Catalog()
    log("loading the resident systems")
    cat.preload(W.serving_queries(2000, rate=max(rates), seed=100))
    warm = W.serving_queries(16, rate=1000.0, seed=99)
    Server(cat, slots=args.slots).serve(warm, time_scale=0.0)
    per_rate = []
    modes = {"on": [True], "off": [False], "both": [True, False]}[args.serve_batch]
    unbatched = []
    for rate in rates:
        count = int(min(2000, max(20, round(rate * args.seconds))))
        qs = W.serving_queries(count, rate=rate, seed=100)
        for batch in modes:
            log(f"rate {rate}/s: {count} queries, batching {'on' if batch else 'off'}")
            res = Server(cat, slots=args.slots, batch=batch).serve(qs)
            s = summarize(res)
            s["rate"] = rate
            s["batch"] = batch
            s["fp32_share"] = sum(q.precision == "fp32" for q in qs) / count
            (per_rate if batch == modes[0] else unbatched).append(s)
            log(f"  p50 {s['p50_ms']:.1f} ms  p99 {s['p99_ms']:.1f} ms  {s['verified_steps_per_s']:.0f} steps/s"
                f"  mean group {s['mean_group']:.2f}")
    top = per_rate[-1]
    out = {
        "metric": "Krylov step HBM GB/s (% peak); verified time-steps/s vs plain FP64; p99 query latency",
        "value": top["verified_steps_per_s"], "unit": "verified time-steps/s", "n_gpus": 1,
        "steps": sum(s["queries"] for s in per_rate), "warmup": len(warm), "ms_per_step": top["p50_ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64+f32-storage",
        "data": "synthetic",
        "config": {"workload": "serving stream: heat / conv-diff queries, n in 1e3..1e7 (13 resident grids), "
                               "1-8 generators, 1-4 outputs, 100-2000 steps, FP64 or FP32 basis, Poisson "
                               f"arrivals, {args.slots} slots", "rates": rates, "seconds_per_rate": args.seconds},
        "latency": per_rate, "latency_unbatched": unbatched or None,
        "resident_system_bytes": cat.resident_bytes(),
    }
    print(json.dumps(out))


def lp_sets(p):
    """The LP bench's sets: the generator box cut by sum_j (z_j - zc_j) / r_j
    <= d / 2 (a polytope), and the conjunction of every output row's
    unsafe interval (its finite ends as halfspaces)."""
    import numpy as np
    zc = np.array([g.zc for g in p.gens]); r = np.array([g.radius for g in p.gens])
    d = len(p.gens)
    live = r > 0
    G = np.zeros((1, d)); G[0, live] = 1.0 / r[live]
    h = np.array([float(G[0] @ zc) + d / 2.0])
    U, u = [], []
    for q, (lo, hi) in enumerate(p.unsafe):
        e = np.zeros(p.o); e[q] = 1.0
        if np.isfinite(hi): U.append(e); u.append(hi)
        if np.isfinite(lo): U.append(-e); u.append(-lo)
    return G, h, np.array(U).reshape(-1, p.o), np.array(u)


def measure(torch, kry, p, dsys, precision, steps, warmup, method=0, error_target=0.0, kernel_events=True,
            transposed=False, check="box", graph=False):
    """Times `steps` whole verifications (after `warmup`), then the same with
    per-kernel HIP events; returns the throughput and per-kernel figures.
    graph: one plan made before the timed region, its projection replayed
    as a HIP graph each step (on a stream of its own)."""
    stream = torch.cuda.Stream() if graph else torch.cuda.current_stream()
    if graph:
        torch.cuda.set_stream(stream)
    used = {}
    krylov_runs = {}
    graph_plan = None
    if graph:
        graph_plan = (kry.TransposedPlan(dsys, stream=stream, precision=precision, method=method) if transposed
                      else kry.Plan(dsys, stream=stream, precision=precision, method=method))
        graph_plan.set_graph(True)
        krylov_runs["n"] = len(graph_plan.runs) if transposed else graph_plan.nruns

    def step():
        if graph_plan is not None:
            graph_plan.project_expm(None)
            v = graph_plan.check_lp(*lp_sets(p)) if check == "lp" else graph_plan.check(p.unsafe)
            return v, graph_plan.nruns
        if transposed:
            plan = kry.TransposedPlan(dsys, stream=stream, precision=precision, method=method)
            krylov_runs["n"] = len(plan.runs)
        else:
            plan = kry.Plan(dsys, stream=stream, precision=precision, method=method)
            krylov_runs["n"] = plan.nruns
        if error_target > 0.0:
            plan.set_error_target(error_target)
        plan.project_expm(None)
        if check == "lp":
            v = plan.check_lp(*lp_sets(p))
            v["row"] = -1
        else:
            v = plan.check(p.unsafe)
        nr = plan.nruns
        if error_target > 0.0 and not used:
            used["k_used"] = [plan.error(r)[0] for r in range(nr)]
            used["bound"] = [plan.error(r)[1] for r in range(nr)]
        plan.close()
        return v, nr

    log(f"warmup {warmup} (precision {precision})")
    for _ in range(warmup):
        verdict, nruns = step()
    torch.cuda.synchronize()
    # timed region 1: the whole job, no instrumentation -> value
    log(f"timing {steps} steps")
    t0 = time.perf_counter()
    for _ in range(steps):
        verdict, nruns = step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    # timed region 2: the same steps with every kernel launch bracketed by HIP
    # events on the plan's stream -> per-kernel durations for the roofline
    elapsed_ev = float("nan")
    if kernel_events:
        log(f"timing {steps} steps with per-kernel events")
        kry.profile_enable(True)
        kry.profile_reset()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(steps):
            verdict, nruns = step()
        torch.cuda.synchronize()
        elapsed_ev = time.perf_counter() - t1
        kry.profile_enable(False)
    if graph_plan is not None:
        graph_plan.close()
        torch.cuda.set_stream(torch.cuda.default_stream())
    kern = {}
    for name in kry.profile_names():
        cnt, ms = kry.profile_read(name)
        if cnt:
            kern[name] = {"launches": cnt, "avg_us": 1000.0 * ms / cnt, "total_ms_per_step": ms / steps}
    # algorithmic bytes per launch, all runs of the plan advanced by one launch
    # (P = runs per batch; every workload here fits one batch)
    es = 4 if precision == kry.KRY_FP32_BASIS else 8
    n, nnz, P, k = p.n, p.nnz, krylov_runs["n"], p.k
    vec = es * n * P
    if p.kind == "csr":
        mat = (4 if es == 4 else 8) * nnz + 4 * nnz + 8 * (n + 1)   # values, int32 columns, int64 row pointers
    else:
        mat = 0                                                   # matrix-free
    lanczos = p.symmetric
    gs = os.environ.get("KRY_ARN_GS", "-1")
    arn_twins = 2 if (not lanczos and (gs == "1" or (gs != "0" and n >= 65536))) else 1
    # the sliced-ELL copy: values and int32 columns of the nnz entries, 12
    # bytes of slice offset and width per 64 rows (padding is not counted)
    mat_sell = ((4 if es == 4 else 8) + 4) * nnz + 12 * (-(-n // 64)) if p.kind == "csr" else 0
    per_launch = {
        "spmv_csr": mat + (3 if lanczos else 2) * vec,        # read v_j (and v_{j-1}), write w
        "spmv_sell": mat_sell + (3 if lanczos else 2) * vec,
        "spmv_stencil": (3 if lanczos else 2) * vec,
        "sweep": 3 * vec,                                     # read v_j, w; write w
        "start": vec,                                         # write u_1
        # classical Gram-Schmidt passes over the stored basis, averaged over
        # iterations j = 1..k (j stored vectors read per pass); with the second
        # pass from the Gram matrix every real launch has a conditional twin
        # that returns at once, so the bytes per launch halve
        "arn_dots": vec * (1 + (k + 1) / 2.0) / arn_twins,
        "arn_update": vec * (2 + (k + 1) / 2.0) / arn_twins,
        # one-pass step: read the pair (u_{j-1}, r_j), write (u_j, r_{j+1});
        # the first of the k launches reads the plain start vectors (one
        # vector), so the average over a batch's launches is (4k - 1)/k
        "lz1_sell": mat_sell + (4 * k - 1) / k * vec,
        "lz1_stencil": (4 * k - 1) / k * vec,
        "lz1_march": (4 * k - 1) / k * vec,
        "lz1_close": 0,                                       # one workgroup: scalars only
    }
    for name, b in per_launch.items():
        if name in kern:
            kern[name]["bytes"] = b
            kern[name]["GBps"] = b / (kern[name]["avg_us"] * 1e-6) / 1e9
    if method == kry.KRY_BLOCK_ARNOLDI:
        # per whole block run: bytes each kernel must move, summed over its
        # launches (16-wide blocks of es-byte entries, n rows)
        blk = 16 * es * n
        tot = {"bspmm": 0.0, "bgram": 0.0, "bupdate": 0.0, "bstart": blk}
        tot["bgram"] += 2 * blk                      # start block CholQR2: Gram of V_1
        tot["bupdate"] += 2 * 2 * blk                # and V_1 R^{-1} in place
        # the default step takes the second Gram-Schmidt pass from the Gram
        # matrix (one pass over V_1..V_j and W for the coefficients, one for
        # the update); KRY_BLOCK_GS=0 makes both passes over the basis.  The
        # conditional second pass (only after a projection that cancels) is
        # not counted: its launches return at once otherwise.
        passes = (1,) if os.environ.get("KRY_BLOCK_GS", "1") != "0" else (1, 2)
        for j in range(1, k + 1):
            tot["bspmm"] += mat + 2 * blk            # A, V_j streamed once, W written
            for ps in passes:
                tot["bgram"] += (j + 1) * blk        # V_1..V_j and W
                if j < k or (ps == 1 and len(passes) == 2):
                    tot["bupdate"] += (j + 2) * blk  # V_1..V_j, W read, W written
            if j < k:
                tot["bgram"] += 2 * blk
                tot["bupdate"] += 2 * 2 * blk
        nblk = -(-len(p.gens) // 16)
        for name, b in tot.items():
            if name in kern:
                kern[name]["bytes"] = b * nblk / max(kern[name]["launches"] / steps, 1)
                kern[name]["GBps"] = kern[name]["bytes"] / (kern[name]["avg_us"] * 1e-6) / 1e9
        dom_name = max((n_ for n_ in ("bgram", "bupdate", "bspmm") if n_ in kern),
                       key=lambda n_: kern[n_]["total_ms_per_step"], default="bgram")
        return {"value": (p.steps + 1) * nruns / (elapsed / steps), "ms_per_step": 1000.0 * elapsed / steps,
                "ms_per_step_ev": 1000.0 * elapsed_ev / steps, "kern": kern, "nruns": nruns, "verdict": verdict,
                "dom_name": dom_name, "error_control": used or None, "krylov_runs": krylov_runs["n"]}
    if p.kind == "csr":
        mv = next((n_ for n_ in ("lz1_sell", "spmv_sell", "spmv_csr") if n_ in kern), "spmv_csr")
    else:
        mv = next((n_ for n_ in ("lz1_march", "lz1_stencil", "spmv_stencil") if n_ in kern), "spmv_stencil")
    # the roofline kernel: the mat-vec, or the one with the most time when a
    # stored-basis pass outweighs it
    dom_name = mv
    for name in ("arn_update", "arn_dots"):
        if name in kern and kern[name]["total_ms_per_step"] > kern.get(dom_name, {}).get("total_ms_per_step", 0):
            dom_name = name
    return {"value": (p.steps + 1) * nruns / (elapsed / steps), "ms_per_step": 1000.0 * elapsed / steps,
            "ms_per_step_ev": 1000.0 * elapsed_ev / steps, "kern": kern, "nruns": nruns, "verdict": verdict,
            "dom_name": dom_name, "error_control": used or None, "krylov_runs": krylov_runs["n"]}


def describe(p, nruns, precision, method_name="auto"):
    prec = "FP64" if precision == "fp64" else "FP32 basis (FP64 sums), full reorthogonalisation"
    if p.name == "conv_diff3d":
        g = p.meta["grid"]
        meth = "block Arnoldi p=16" if method_name == "block" else "Arnoldi"
        return (f"3D convection-diffusion {g[0]}x{g[1]}x{g[2]} CSR (n={p.n}, nnz={p.nnz}, nonsymmetric), "
                f"{len(p.gens)} generators, {meth}, k={p.k}, dt={p.dt}, {p.steps} steps, o={p.o}, {prec}")
    if p.name == "heat3d_csr":
        m = p.meta["m"]
        return (f"3D heat {m}^3 CSR (n={p.n}, nnz={p.nnz}) + affine forcing, Lanczos k={p.k}, dt={p.dt}, "
                f"{p.steps} steps, o={p.o}, runs={nruns}, {prec}")
    if p.name == "heat3d_stencil":
        m = p.meta["m"]
        return (f"3D heat {m}^3 matrix-free 7-point (n={p.n}) + affine forcing, Lanczos k={p.k}, dt={p.dt}, "
                f"{p.steps} steps, o={p.o}, runs={nruns}, {prec}")
    if p.name == "heat3d_paper_stencil":
        m = p.meta["m"]
        return (f"3D heat {m}^3 as in the paper (insulated faces, exchange 0.5 at x=1, matrix-free n={p.n}), "
                f"centre-point output, three-vector Lanczos k={p.k}, dt={p.dt}, {p.steps} steps, {prec}")
    if p.name == "heat3d_paper":
        m = p.meta["m"]
        return (f"3D heat {m}^3 as in the paper (insulated faces, exchange 0.5 at x=1, CSR n={p.n}, nnz={p.nnz}), "
                f"centre-point output, three-vector Lanczos with the Lemma 1 error control (k <= {p.k}), "
                f"dt={p.dt}, {p.steps} steps, {prec}")
    if p.name in ("heat3d_many_inputs", "heat3d_many_gens"):
        m = p.meta["m"]
        return (f"3D heat {m}^3 CSR (n={p.n}, nnz={p.nnz}) + forcing, {len(p.gens)} generators + center + forcing = "
                f"{nruns} basis columns, o={p.o} output, Lanczos k={p.k}, dt={p.dt}, {p.steps} steps, {prec}")
    return f"{p.name} n={p.n} nnz={p.nnz} k={p.k} dt={p.dt} steps={p.steps} o={p.o} runs={nruns} {prec}"


def counter_traffic(path, sources):
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
        h = hashlib.sha256()
        for f in sources:
            h.update(open(os.path.join(ROOT, "paper_1804_01583_amd", "csrc", f), "rb").read())
        if h.hexdigest() != vals["kernel_source_sha256"]:
            return None
        rd = float(vals["fetch_kib_per_launch"]) * 1024 * float(vals["calib_read_factor"])
        wr = float(vals["write_kib_per_launch"]) * 1024 * float(vals["calib_write_factor"])
        return rd + wr
    except (KeyError, ValueError):
        return None


def basis_of(kry, dsys, precision, method):
    """One verification's basis (steps+1, o, columns) on the host."""
    plan = kry.Plan(dsys, precision=precision, method=method)
    b = plan.basis()
    plan.close()
    return b


def per_output_error(b, ref):
    """Per (output row, basis column): max over steps of |b - ref| divided by
    max over steps of |ref| (0 where both are exactly zero)."""
    import numpy as np
    out = []
    for q in range(ref.shape[1]):
        row = []
        for r in range(ref.shape[2]):
            scale = float(np.abs(ref[:, q, r]).max())
            err = float(np.abs(b[:, q, r] - ref[:, q, r]).max())
            row.append(err / scale if scale > 0 else (0.0 if err == 0.0 else float("inf")))
        out.append(row)
    return out


def fp32_side_measure(torch, kry, p, dsys, m64, method, steps=3, warmup=1):
    """The FP32-basis mode on the same workload (a few timed verifications):
    its throughput against the FP64 line and the error of every output
    against the FP64 basis."""
    m32 = measure(torch, kry, p, dsys, kry.KRY_FP32_BASIS, steps, warmup, method, kernel_events=False)
    torch.cuda.empty_cache()
    b32 = basis_of(kry, dsys, kry.KRY_FP32_BASIS, method)
    torch.cuda.empty_cache()
    b64 = basis_of(kry, dsys, kry.KRY_FP64, method)
    torch.cuda.empty_cache()
    return {"value": m32["value"], "unit": "verified time-steps/s", "ms_per_step": m32["ms_per_step"],
            "steps": steps, "warmup": warmup, "ratio_over_fp64": m32["value"] / m64["value"],
            "max_rel_err_per_output": per_output_error(b32, b64),
            "error_definition": "per (output row, basis column): max over steps of |FP32-basis - FP64| / "
                                "max over steps of |FP64| (0 where both are exactly zero)",
            "verdict": {"first_step": m32["verdict"]["first_step"], "row": m32["verdict"]["row"]}}


def host_cores():
    """Physical cores this process may use, at most 16 (one GPU's share of
    the host)."""
    try:
        import psutil
        phys = psutil.cpu_count(logical=False) or 1
    except Exception:   # pragma: no cover
        phys = os.cpu_count() or 1
    return max(1, min(phys, len(os.sched_getaffinity(0)), 16))


def cpu_baseline_subgrids(p):
    """The oracle on the matrix-free heat system through its locality
    sub-grids: every run of the 1000^3 system equals the same run on the
    sub-grid of its start box dilated by k + 1 cells (outputs outside it are
    exactly zero), so the oracle computes the whole verification's basis
    from those.  Timed at one thread and at the host's physical cores."""
    try:
        from threadpoolctl import threadpool_limits
    except Exception:   # pragma: no cover
        threadpool_limits = None
    import contextlib
    import oracle
    import workloads as W
    roles = ["gen", "affine"] if p.has_forcing else ["gen"]
    subs = [(role, W.heat3d_stencil_subgrid(p, role)[0]) for role in roles]
    live = [sub for _, sub in subs if sub is not None]

    def run(threads):
        ctx = threadpool_limits(limits=threads) if threadpool_limits else contextlib.nullcontext()
        with ctx:
            t0 = time.perf_counter()
            for sub in live:
                oracle.verify(sub)
            return time.perf_counter() - t0

    cores = host_cores()
    t1 = run(1)
    tc = run(cores) if cores > 1 else t1
    cols = len(roles)
    desc = ", ".join(f"{role}: {'sub-grid ' + 'x'.join(map(str, sub.grid)) + f' ({sub.n} states)' if sub else 'no output within reach, exactly zero'}"
                     for role, sub in subs)
    return {"value": (p.steps + 1) * cols / tc, "unit": "verified time-steps/s", "cores": cores, "kind": "oracle",
            "sample": f"the whole verification's basis ({cols} columns x {p.steps + 1} time points) by the oracle "
                      f"on the locality sub-grids ({desc}); {tc:.1f} s at {cores} threads",
            "single_thread": {"value": (p.steps + 1) * cols / t1, "cores": 1, "seconds": t1}}


def cpu_baseline(p, transposed=False, check="box"):
    """The oracle as it stands, on this host's CPU, one thread, over one whole
    verification of the same workload (by the same route and check)."""
    try:
        from threadpoolctl import threadpool_limits
    except Exception:   # pragma: no cover
        threadpool_limits = None
    import oracle
    import oracle.lp
    import oracle.transpose
    route = oracle.transpose.verify_transposed if transposed else oracle.verify

    def verify(p):
        res = route(p)
        if check == "lp":
            zc = [g.zc for g in p.gens]; r = [g.radius for g in p.gens]
            res["lp"] = oracle.lp.lp_check(res["basis"], res["roles"], zc, r, *lp_sets(p))
        return res
    t0 = time.perf_counter()
    if threadpool_limits is not None:
        with threadpool_limits(limits=1):
            res = verify(p)
    else:
        res = verify(p)
    dt = time.perf_counter() - t0
    nruns = res["basis"].shape[2]
    return {"value": (p.steps + 1) * nruns / dt, "unit": "verified time-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"one whole verification of the same workload ({dt:.1f} s, {nruns} runs, "
                      f"{p.steps + 1} time points)"}


if __name__ == "__main__":
    main()
