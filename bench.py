#!/usr/bin/env python3
"""Time to a 1e-8 relative nonlinear residual for one implicit VP momentum step.

One "step" is a whole stress-velocity Newton solve (residual, assembly, AMG
setup, AMG-preconditioned Krylov, energy backtracking, dual update; Sec. 4.2,
5.1, 5.4) from v = 0, pi = 0 on the 2048 x 2048 Q1 workload (8,396,802
unknowns; wind to 25 m/s, H in [0.05, 1.5] m, Delta_min = 2e-10).  Inputs are
resident in HBM before the timed region.  Paths: plain FP64; FP32 V-cycle and
preconditioner SpMV; FP32 V-cycle with BF16 coarse-level storage (the mixed
mode); each mixed mode also from the learned start (U-Net inference and the
energy choice inside the timed region).  Residual, tau/Delta, Krylov
orthogonalisation and update are FP64 in every path.  `value` is the mixed +
learned path's time, reported beside plain FP64; every path's final velocity is
compared with the FP64 path's and put through the CPU oracle's residual.

Prints exactly one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PREC = {"fp64": 0, "fp32": 1, "fp32+learned": 1, "bf16": 2, "bf16+learned": 2, "bf16all": 3, "bf16all+learned": 3,
        "fp16": 4, "fp16+learned": 4, "fp16all": 5, "fp16all+learned": 5, "fp16c32": 6, "fp16c32+learned": 6}
METRIC = "time-to-1e-8 residual, 2048^2 mesh: plain FP64 vs mixed+learned; SpMV GB/s"
HEADLINE = "bf16+learned"   # FP32 V-cycle, BF16 coarse storage, learned start
HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0   # dense BF16 matrix-core peak


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def cpu_baseline(samples, gpu_newton_its: int, n_full: int):
    """The CPU oracle on a bounded sample: full Newton solves (direct inner solves,
    one thread) of the same recipe on the meshes in `samples`.  The time per Newton
    iteration is fitted as a * unknowns^p through the measured meshes and
    extrapolated to the full mesh, times the GPU's Newton iteration count there."""
    import math

    from threadpoolctl import threadpool_limits

    from oracle import vp_oracle as O
    from paper_2204_10822_amd import inputs

    meas = []
    for ns in samples:
        w = inputs.sharp_step(ns)
        prob = O.problem_from_workload(w)
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            res = O.newton_solve(prob, tol=1e-8, maxit=200)
            t = time.perf_counter() - t0
        meas.append(dict(n=ns, dofs=2 * (ns + 1) ** 2, seconds=t, newton_its=res.iterations,
                         converged=res.converged, s_per_it=t / max(res.iterations, 1)))
        log(f"cpu baseline: oracle {ns}^2: {t:.2f} s, {res.iterations} Newton its")
    a, b = meas[0], meas[-1]
    p = math.log(b["s_per_it"] / a["s_per_it"]) / math.log(b["dofs"] / a["dofs"]) if len(meas) > 1 else 1.0
    dofs_f = 2 * (n_full + 1) ** 2
    per_it = b["s_per_it"] * (dofs_f / b["dofs"]) ** p
    return dict(value=per_it * gpu_newton_its, unit="s", cores=1, kind="oracle",
                sample=("oracle Newton solves (direct sparse inner solves, 1 thread) of the same recipe on "
                        + ", ".join(f"{m['n']}^2 ({m['seconds']:.1f} s, {m['newton_its']} its)" for m in meas)
                        + f"; time per Newton iteration ~ unknowns^{p:.2f} fitted through them, "
                        f"extrapolated to {n_full}^2 and multiplied by the GPU's {gpu_newton_its} Newton its"),
                measured=meas, exponent=p, sample_seconds=sum(m["seconds"] for m in meas))


def _oracle_rel_residual(args):
    """||R(v)|| / ||R(0)|| of the oracle's residual (eq. A - eq. F) at a GPU
    solution v of the n^2 benchmark recipe (runs in a worker process)."""
    import numpy as np

    from oracle import vp_oracle as O
    from paper_2204_10822_amd import inputs

    n, v = args
    prob = O.problem_from_workload(inputs.sharp_step(n))
    r = np.linalg.norm(prob.residual(v))
    r0 = np.linalg.norm(prob.residual(np.zeros_like(v)))
    return float(r / r0)


def oracle_residuals(n, vs):
    """The oracle's relative residual at each path's final velocity, in parallel
    worker processes (fresh interpreters: they never touch the GPU)."""
    import concurrent.futures as cf
    import multiprocessing as mp

    names = list(vs)
    workers = min(len(names), 6)
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        out = list(ex.map(_oracle_rel_residual, [(n, vs[k]) for k in names]))
    return dict(zip(names, out))


PROFILES = os.path.join(ROOT, "profiles")
CALIB_READ_KIB, CALIB_WRITE_KIB = 2 << 20, 1 << 20   # the triad of kernel_sequence


def counter_traffic(kernel_name):
    """HBM bytes per launch of `kernel_name` from the committed counter summaries:
    (traffic, FETCH_SIZE + WRITE_SIZE as read).  Traffic counts every L2->memory
    request at its own size (128/64/32-B reads, 64/32-B writes) from the
    size-split request counters; without that summary it falls back to the
    FETCH_SIZE/WRITE_SIZE pair scaled by their reading for the calibration triad
    (FETCH_SIZE counts a 128-B read request as 64 B).  (None, None) if the kernel
    is missing."""
    def table(fname, col):
        path = os.path.join(PROFILES, fname)
        if not os.path.exists(path):
            return None
        rows = {}
        for line in open(path):
            if line.startswith("#") or not line.strip():
                continue
            parts = line.rsplit(None, col)
            if len(parts) == col + 1 and parts[1].isdigit():
                try:
                    rows[parts[0].strip()] = [float(x) for x in parts[2:]]
                except ValueError:
                    pass
        return rows
    fetch = table("vp_sharp_2048_kernels_fetch_size.txt", 3)
    write = table("vp_sharp_2048_kernels_write_size.txt", 3)
    raw = None
    if fetch and write and kernel_name in fetch and kernel_name in write:
        raw = 1024.0 * (fetch[kernel_name][0] + write[kernel_name][0])
    req = table("vp_sharp_2048_kernels_requests.txt", 10)
    if req and kernel_name in req:
        return 1e6 * req[kernel_name][7], raw   # total_MB column
    if raw is None:
        return None, None
    cal_f = max(v[0] for k, v in fetch.items() if "elementwise" in k)
    cal_w = max(v[0] for k, v in write.items() if "elementwise" in k)
    calibrated = 1024.0 * (fetch[kernel_name][0] * CALIB_READ_KIB / cal_f +
                           write[kernel_name][0] * CALIB_WRITE_KIB / cal_w)
    return calibrated, raw


_STORAGE = {"fp64": ("double", "double"), "fp32": ("float", "float"), "fp16": ("_Float16", "float"),
            "bf16": ("__hip_bfloat16", "float")}


def kernel_name(kid, kind):
    """Name in the rocprofv3 summaries of the kernel behind a profiled kernel id."""
    tm, tv = _STORAGE[kind]
    return {"apply_fine": "k_apply_fine<2, 4>",
            "cheb_step0": f"k_cheb_step<2, {tm}, {tv}, 0>",
            "sten_resid0": f"k_sten_resid<2, {tm}, {tv}, 0>",
            "cheb_pair0": (f"k_cheb_walk<0, 0, {tv}, {12 if tv == 'double' else 10}>" if tm == tv
                           else f"k_cheb_pair<0, 0, {tm}, {tv}, 62, 14, 1024, 4>"),
            "cheb_walk4": f"k_cheb_walk4<0, {tv}>",
            "residual": "k_residual",
            "assemble": "k_assemble"}.get(kid)


def dtype_of(path):
    """Arithmetic types a path computes in: the V-cycle's storage and arithmetic, plus
    BF16 for the learned start's network."""
    t = {0: "f64", 1: "f64+f32", 2: "f64+f32+bf16", 3: "f64+f32+bf16", 4: "f64+f32+fp16+bf16",
         5: "f64+f32+fp16", 6: "f64+f32+fp16"}[PREC[path]]
    if path.endswith("learned") and "bf16" not in t:
        t += "+bf16"
    return t


def storage_kind(path):
    """Finest-level operator storage of a benchmark path."""
    p = PREC[path]
    return "fp64" if p == 0 else "fp32" if p in (1, 2) else "bf16" if p == 3 else "fp16"


def kernel_sequence(args, ctx, v, pi, torch, vp):
    """Short fixed launch sequence for profiler passes: three Newton steps (to get
    a non-trivial operator), then per path 10 V-cycles and 10 FP64 operator
    products, and a 1 GiB device copy whose counters calibrate the byte counters."""
    no, ao, ko = vp.default_opts()
    for k in range(3):
        rc, info = ctx.vp_newton_step(v, pi, no, ao, ko)
        log(f"newton step {k}: rc={rc} rel={info.rnorm_new / info.rnorm0:.2e}")
    r = torch.randn_like(v)
    z = torch.zeros_like(v)
    for path in [p for p in args.paths.split(",") if p]:
        ao.precision = PREC[path]
        ctx.vp_amg_setup(ao)
        for _ in range(10):
            ctx.vp_amg_apply(r, z)
        for _ in range(10):
            ctx.vp_operator_apply(r, z)
        torch.cuda.synchronize()
        log(f"{path}: 10 V-cycles and 10 operator products done")
    # calibration for the byte counters: a triad of known size (reads 2 GiB,
    # writes 1 GiB), the largest elementwise dispatch of this sequence
    a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    b = torch.ones_like(a)
    c = torch.empty_like(a)
    torch.add(a, b, alpha=0.5, out=c)
    torch.cuda.synchronize()
    log("calibration triad (2 GiB read, 1 GiB written) done")
    c.copy_(a)                                   # a plain 1 GiB device copy, for comparison
    torch.cuda.synchronize()
    log("device copy (1 GiB read, 1 GiB written) done")
    print(json.dumps({"mode": "kernels", "paths": args.paths, "n": args.n}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--paths", default="fp64,fp32,fp32+learned,bf16,bf16+learned",
                    help="comma list of fp64, fp32, fp32+learned, bf16, bf16+learned, bf16all, bf16all+learned, fp16, fp16+learned, fp16all, "
                         "fp16all+learned, fp16c32 (FP16 finest, FP32 coarse), fp16c32+learned")
    ap.add_argument("--cpu-samples", default="128,192",
                    help="meshes of the oracle's bounded CPU sample (comma list)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-oracle-check", action="store_true",
                    help="skip the oracle's residual at each path's final velocity")
    ap.add_argument("--mode", default="solve", choices=["solve", "kernels"],
                    help="kernels: a short fixed sequence (for profiler counter passes)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the solver has no multi-GPU path "
              "(a single-GPU implementation; the mesh would shard by row strips with halo exchange).",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2204_10822_amd import inputs, vp

    torch.cuda.set_device(0)
    n = args.n
    t0 = time.time()
    w = inputs.sharp_step(n)
    ctx = vp.context_for(w)
    log(f"workload {w.name}: {2 * (n + 1) ** 2} unknowns, inputs ready in {time.time() - t0:.1f}s")
    nn = (n + 1) ** 2
    v = torch.zeros(nn, 2, dtype=torch.float64, device="cuda")
    pi = torch.zeros(4, 3, n, n, dtype=torch.float64, device="cuda")

    if args.mode == "kernels":
        return kernel_sequence(args, ctx, v, pi, torch, vp)

    def opts(path):
        no, ao, ko = vp.default_opts()
        ao.precision = PREC[path]
        return no, ao, ko

    ws = None
    if any(p.endswith("learned") for p in args.paths.split(",")):
        from paper_2204_10822_amd import warmstart
        if os.path.exists(warmstart.WEIGHTS):
            ws = warmstart.WarmStart()
        else:
            log("no trained warm-start weights: skipping the learned path")
            args.paths = ",".join(p for p in args.paths.split(",") if not p.endswith("learned"))
    starts = {}

    def solve(path):
        no, ao, ko = opts(path)
        if path.endswith("learned"):
            # learned start (U-Net on the pooled 256-cell grid) chosen against the
            # zero start by energy, and a rerun from zero if Newton fails from it;
            # all inside the timed region
            rc, info, starts[path] = warmstart.solve_with_fallback(ctx, ws, v, pi, ("learned", "zero"), no, ao, ko)
            return rc, info
        v.zero_()
        pi.zero_()
        rc, info, _ = ctx.vp_newton_solve(v, pi, 200, no, ao, ko, history=False)
        return rc, info

    results = {}
    finals = {}
    for path in [p for p in args.paths.split(",") if p]:
        for k in range(args.warmup):
            rc, info = solve(path)
            log(f"{path} warmup {k}: rc={rc} newton={info.iterations} krylov={info.krylov_iters} "
                f"rel={info.rel_resid:.2e}")
        torch.cuda.synchronize()
        ctx.vp_profile(1)
        times, infos = [], []
        torch.cuda.synchronize()
        tstart = time.perf_counter()
        for k in range(args.steps):
            ts = time.perf_counter()
            rc, info = solve(path)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - ts)
            infos.append(info)
            if rc != 0 or info.rel_resid > 1e-8:
                raise SystemExit(f"{path} solve failed: rc={rc} rel={info.rel_resid:.2e}")
            log(f"{path} step {k}: {times[-1]:.3f}s newton={info.iterations} "
                f"krylov={info.krylov_iters} rel={info.rel_resid:.2e}")
        torch.cuda.synchronize()
        total = time.perf_counter() - tstart
        ctx.vp_profile(0)
        kern = {}
        for name, kid in vp.VP_KID.items():
            ms, cnt, b = ctx.vp_profile_read(kid)
            if cnt:
                kern[name] = dict(total_ms=ms, launches=cnt, avg_us=1e3 * ms / cnt,
                                  bytes_per_launch=b,
                                  gbs=(b / (ms / cnt * 1e-3) / 1e9) if b > 0 and ms > 0 else None)
        results[path] = dict(total=total, times=times, median=statistics.median(times),
                             newton=[i.iterations for i in infos],
                             krylov=[i.krylov_iters for i in infos], kernels=kern,
                             rel_resid=infos[-1].rel_resid)
        finals[path] = v.detach().cpu().numpy().ravel().copy()

    # every path's final velocity against the plain FP64 path's (host, after the
    # timed regions)
    import numpy as np
    if "fp64" in finals:
        ref = finals["fp64"]
        for p_, vv in finals.items():
            results[p_]["rel_l2_vs_fp64"] = float(np.linalg.norm(vv - ref) / np.linalg.norm(ref))

    # headline: the mixed-precision + learned-start path the metric names, beside
    # plain FP64 (both reported); otherwise the fastest path
    best = HEADLINE if HEADLINE in results else min(results, key=lambda p: results[p]["median"])
    fastest = min(results, key=lambda p: results[p]["median"])
    R = results[best]
    # dominant single kernel (by summed time) of the headline path
    single = {k: d for k, d in R["kernels"].items() if k != "vcycle" and d["bytes_per_launch"] > 0}
    dom = max(single, key=lambda k: single[k]["total_ms"])
    D = single[dom]
    kname = kernel_name(dom, storage_kind(best))
    traffic, traffic_raw = counter_traffic(kname) if kname else (None, None)
    roof = dict(kernel=kname or dom, bound="hbm", achieved=D["gbs"], peak=HBM_PEAK_GBS, unit="GB/s",
                frac=D["gbs"] / HBM_PEAK_GBS, traffic=traffic, traffic_fetch_write_size=traffic_raw,
                bytes_per_launch=D["bytes_per_launch"], avg_us=D["avg_us"])
    spmv = R["kernels"].get("apply_fine")
    out = {
        "metric": METRIC,
        "value": R["median"],
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * R["total"] / args.steps,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype_of(best),
        "data": "synthetic",
        "config": {"workload": w.name, "mesh": f"{n}x{n} Q1", "unknowns": 2 * nn,
                   "tol": 1e-8, "path": best, "newton_its": R["newton"], "krylov_its": R["krylov"],
                   "fp64_s": results["fp64"]["median"] if "fp64" in results else None,
                   "speedup_vs_fp64": (results["fp64"]["median"] / R["median"]) if "fp64" in results else None,
                   "fastest_path": fastest},
        "paths": {p: dict(median_s=d["median"], times_s=d["times"], newton_its=d["newton"],
                          krylov_its=d["krylov"], start=starts.get(p, "zero"), rel_resid=d["rel_resid"],
                          rel_l2_vs_fp64=d.get("rel_l2_vs_fp64"), oracle_rel_resid=None)
                  for p, d in results.items()},
        "spmv_gbs": spmv["gbs"] if spmv else None,
        "kernels": R["kernels"],
        "roofline": roof,
    }
    # achievable streaming bandwidth on this device: a 1 GiB device copy and a triad
    a_ = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    b_ = torch.ones_like(a_)
    c_ = torch.empty_like(a_)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    stream = {}
    for name, fn, nbytes in (("copy", lambda: c_.copy_(a_), 2 << 30),
                             ("triad", lambda: torch.add(a_, b_, alpha=0.5, out=c_), 3 << 30)):
        fn()
        torch.cuda.synchronize()
        ev0.record()
        for _ in range(10):
            fn()
        ev1.record()
        torch.cuda.synchronize()
        stream[name + "_gbs"] = nbytes / (ev0.elapsed_time(ev1) / 10 * 1e-3) / 1e9
    del a_, b_, c_
    out["stream"] = stream
    out["roofline"]["frac_of_measured_triad"] = D["gbs"] / stream["triad_gbs"]
    log(f"stream: copy {stream['copy_gbs']:.0f} GB/s, triad {stream['triad_gbs']:.0f} GB/s")
    # learned warm start kernels: BF16 MFMA forward and training step on 256^2 inputs
    try:
        from paper_2204_10822_amd import warmstart as _ws
        nb = _ws.bench_net(batch=8, reps=10)
        nb1 = _ws.bench_net(batch=1, reps=20)
        out["unet"] = dict(
            forward_b1_ms=nb1["forward"]["ms"], forward_b8_ms=nb["forward"]["ms"],
            train_step_b8_ms=nb["train_step"]["ms"],
            roofline=dict(kernel="unet train step (all layers)", bound="mfma",
                          achieved=nb["train_step"]["tflops"], peak=BF16_PEAK_TFLOPS, unit="TFLOP/s",
                          frac=nb["train_step"]["tflops"] / BF16_PEAK_TFLOPS),
            forward_tflops=nb["forward"]["tflops"])
        log(f"unet: forward b8 {nb['forward']['ms']:.2f} ms ({nb['forward']['tflops']:.1f} TFLOP/s), "
            f"train step b8 {nb['train_step']['ms']:.2f} ms")
    except Exception as e:  # the solver metric stands on its own
        out["unet"] = dict(error=str(e))
    # the CPU oracle leg: the oracle's residual at every path's final velocity, and
    # the oracle's own time on a bounded sample
    if not args.no_cpu and not args.no_oracle_check:
        t_or = time.time()
        orr = oracle_residuals(n, finals)
        for p_, r_ in orr.items():
            out["paths"][p_]["oracle_rel_resid"] = r_
        log("oracle residual at each path's velocity: "
            + ", ".join(f"{k} {v_:.2e}" for k, v_ in orr.items()) + f" ({time.time() - t_or:.0f}s)")
    if not args.no_cpu:
        samples = [int(x) for x in args.cpu_samples.split(",") if x]
        ref_path = "fp64" if "fp64" in results else best
        log(f"cpu baseline: oracle on {samples} samples")
        out["cpu_baseline"] = cpu_baseline(samples, results[ref_path]["newton"][0], n)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
