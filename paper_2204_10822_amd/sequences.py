"""Sequences of implicit momentum steps on the GPU path (Sec. 3: one implicit
Euler step per dt, each a stress-velocity Newton solve whose previous velocity
is the step before's solution).  A and H stay fixed; the wind's vortices drift
10 m/s (18 km per half-hour step); step k takes the wind at (k - 1) dt.

  c2: 512^2 cells, seed 2, 10 steps, FP64 end to end.  Reports Newton and Krylov
      iterations per step, Krylov iterations per Newton step, and per-kernel
      durations and GB/s of assembly, residual, the Krylov operator product and
      the V-cycle (the 42 MB FP64 operator fits in the 256 MB Infinity Cache, so
      these rates are cache-resident, not HBM figures).
  c5: 1024^2 cells, seed 5, wind to 25 m/s, 48 steps (one day).  The mixed path
      (FP32 V-cycle, BF16 coarse storage) with the learned start at the first step
      (chosen by energy against the zero start; Newton rerun from zero if it fails
      from the learned start) and the previous step's solution after that, against
      plain FP64 Newton from the previous step.  Reports cumulative solve time, Newton and Krylov iterations and the
      final-step velocity error of the mixed + learned path against the FP64 one.

Timing covers the GPU solve of each step (state upload of the drifted wind,
start selection, Newton), not the host-side generation of the wind field.
One JSON line per run on stdout.

    python -m paper_2204_10822_amd.sequences c2
    python -m paper_2204_10822_amd.sequences c5 [--save FILE.npz]
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

from . import inputs, vp

PREC = {"fp64": vp.VP_PREC_FP64, "fp32": vp.VP_PREC_FP32, "bf16": vp.VP_PREC_FP32_BF16COARSE}


def log(*a):
    print("[sequence]", *a, file=sys.stderr, flush=True)


def run(w0, steps, precision="fp64", learned=False, profile=False, keep_last=False):
    """Run `steps` implicit steps of workload w0 on one context.  Returns a dict of
    per-step statistics, the final (and, with keep_last, the previous) velocity
    on the host, and per-kernel profile data when asked."""
    ctx = vp.Context(w0.desc)
    d = lambda a: vp.to_device(a.reshape(-1, 2) if a.ndim == 3 else a)
    H, A, vo = d(w0.H), d(w0.A), d(w0.v_ocean)
    v = torch.zeros(ctx.node_shape, dtype=torch.float64, device="cuda")
    pi = torch.zeros(ctx.pi_shape, dtype=torch.float64, device="cuda")
    vprev = torch.zeros_like(v)
    no, ao, ko = vp.default_opts()
    ao.precision = PREC[precision]
    ws = None
    if learned:
        from . import warmstart
        ws = warmstart.WarmStart()
    rows = []
    v_before = None
    if profile:
        ctx.vp_profile(1)
    for k in range(1, steps + 1):
        va = d(inputs.sequence_wind(w0, k))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        vprev.copy_(v)
        ctx.vp_set_state(H, A, va, vo, vprev)
        start = "previous" if k > 1 else "zero"
        if ws is not None and k == 1:
            # the learned start from rest; later steps start from the previous
            # step's solution, which beats the network's proposal there
            from . import warmstart
            rc, info, start = warmstart.solve_with_fallback(ctx, ws, v, pi, ("learned", "zero"), no, ao, ko)
        else:
            rc, info, _ = ctx.vp_newton_solve(v, pi, 200, no, ao, ko, history=False)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if rc != 0:
            raise RuntimeError(f"step {k}: solve failed, rc={rc}")
        rows.append(dict(step=k, newton=info.iterations, krylov=info.krylov_iters, seconds=dt, start=start,
                         rel_resid=info.rel_resid))
        if keep_last and k == steps - 1:
            v_before = v.detach().cpu().numpy().ravel().copy()
        log(f"{w0.name} {precision}{'+learned' if learned else ''} step {k}: {dt:.3f}s newton={info.iterations} "
            f"krylov={info.krylov_iters} start={start}")
    kern = {}
    if profile:
        ctx.vp_profile(0)
        for name, kid in vp.VP_KID.items():
            ms, cnt, b = ctx.vp_profile_read(kid)
            if cnt:
                us = 1e3 * ms / cnt
                kern[name] = dict(launches=cnt, avg_us=us, bytes_per_launch=b,
                                  gbs=(b / (us * 1e-6) / 1e9) if b > 0 else None)
    out = dict(rows=rows, v=v.detach().cpu().numpy().ravel(), v_before=v_before, kernels=kern)
    ctx.close()
    return out


def summary(rows):
    nt = sum(r["newton"] for r in rows)
    kt = sum(r["krylov"] for r in rows)
    return dict(seconds=sum(r["seconds"] for r in rows), newton=nt, krylov=kt,
                krylov_per_newton=kt / max(nt, 1), mean_newton=nt / len(rows),
                newton_per_step=[r["newton"] for r in rows], krylov_per_step=[r["krylov"] for r in rows],
                starts=[r["start"] for r in rows])


def c2(steps=10, n=512):
    w0 = inputs.medium_steps(n)
    run(w0, 2, "fp64")                                  # warm-up (code objects, allocations)
    r = run(w0, steps, "fp64", profile=True)
    out = dict(config="c2", workload=w0.name, n=n, steps=steps, path="fp64", **summary(r["rows"]),
               kernels=r["kernels"], cache_resident=True)
    return out, r


def c5(steps=48, n=1024, save=None):
    w0 = inputs.long_run(n)
    run(w0, 2, "fp64")
    ref = run(w0, steps, "fp64", keep_last=save is not None)
    mix = run(w0, steps, "bf16", learned=True, keep_last=save is not None)
    err = float(np.linalg.norm(mix["v"] - ref["v"]) / np.linalg.norm(ref["v"]))
    out = dict(config="c5", workload=w0.name, n=n, steps=steps,
               fp64=summary(ref["rows"]), mixed_learned=summary(mix["rows"]),
               speedup=sum(x["seconds"] for x in ref["rows"]) / sum(x["seconds"] for x in mix["rows"]),
               final_rel_l2_mixed_vs_fp64=err)
    if save:
        np.savez(save, fp64_v=ref["v"], fp64_v_before=ref["v_before"], mixed_v=mix["v"],
                 mixed_v_before=mix["v_before"], n=n, steps=steps)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("config", choices=["c2", "c5"])
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--n", type=int, default=None)
    ap.add_argument("--save", default=None, help="c5: write the last two velocities of both paths here")
    a = ap.parse_args()
    torch.cuda.set_device(0)
    if a.config == "c2":
        out, _ = c2(a.steps or 10, a.n or 512)
    else:
        out = c5(a.steps or 48, a.n or 1024, a.save)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
