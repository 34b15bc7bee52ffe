"""The paper's test problems (Sec. 5.2, 5.3) on the GPU path.

Problem I, the single momentum solve: the stress-velocity Newton method (svN) and
the standard Newton method (stdN) at 1 km, 0.5 km and 0.25 km (512^2, 1024^2,
2048^2 cells) with the paper's stopping rule, a 10^4 reduction of the nonlinear
residual, and a cap of 200 Newton iterations.

Problem II, the time-dependent benchmark: explicit transport of A and H and one
momentum solve per half-hour step, Newton iterations per step averaged over the
run (the quantity of the paper's Table meaniter).

One JSON line per run.

    python -m paper_2204_10822_amd.problems one --n 512,1024,2048 --variants svn,std
    python -m paper_2204_10822_amd.problems two --n 128,256 --steps 192 --variants svn,std
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import torch

from . import inputs, vp

PREC = {"fp64": vp.VP_PREC_FP64, "fp32": vp.VP_PREC_FP32, "bf16": vp.VP_PREC_FP32_BF16COARSE,
        "fp16": vp.VP_PREC_FP16_BF16COARSE, "fp16all": vp.VP_PREC_FP16, "fp16c32": vp.VP_PREC_FP16_FP32COARSE}


def run_problem_one(n: int, variant: str, precision: str = "fp64", tol: float = 1e-4, maxit: int = 200,
                    warmup: bool = True, order: int = 1, amg: str = "sa") -> dict:
    w = inputs.problem_one(n, order)
    ctx = vp.context_for(w)
    v = torch.zeros(ctx.node_shape, dtype=torch.float64, device="cuda")
    pi = torch.zeros(ctx.pi_shape, dtype=torch.float64, device="cuda")
    no, ao, ko = vp.default_opts()
    no.variant = vp.VP_SVN if variant == "svn" else vp.VP_STDN
    no.tol = tol
    ao.precision = PREC[precision]
    ao.kind = vp.VP_AMG_RS if amg == "rs" else vp.VP_AMG_SA

    def solve():
        v.zero_()
        pi.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, info, hist = ctx.vp_newton_solve(v, pi, maxit, no, ao, ko, history=True)
        torch.cuda.synchronize()
        return rc, info, hist, time.perf_counter() - t0

    if warmup:
        solve()
    rc, info, hist, dt = solve()
    ctx.close()
    return dict(problem="problem_one", n=n, order=order, amg=amg, dx_km=512.0 / n, variant=variant,
                precision=precision,
                tol=tol, maxit=maxit, rc=rc, converged=info.rel_resid <= tol,
                newton_its=info.iterations, krylov_its=info.krylov_iters, rel_resid=info.rel_resid,
                seconds=dt, history=[float(h) for h in hist])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("problem", nargs="?", default="one", choices=["one", "two"])
    ap.add_argument("--steps", type=int, default=96, help="Problem II: half-hour steps")
    ap.add_argument("--delta-min", type=float, default=2e-9, help="Problem II")
    ap.add_argument("--n", default="512,1024,2048")
    ap.add_argument("--variants", default="svn,std")
    ap.add_argument("--precision", default="fp64", choices=sorted(PREC))
    ap.add_argument("--tol", type=float, default=1e-4)
    ap.add_argument("--maxit", type=int, default=200)
    ap.add_argument("--no-warmup", action="store_true")
    ap.add_argument("--order", type=int, default=1, choices=[1, 2], help="velocity elements: Q1 or Q2")
    ap.add_argument("--amg", default="sa", choices=["sa", "rs"],
                    help="preconditioner: smoothed aggregation or classical AMG with the paper's settings")
    args = ap.parse_args()
    torch.cuda.set_device(0)
    for n in [int(x) for x in args.n.split(",") if x]:
        for var in [x for x in args.variants.split(",") if x]:
            if args.problem == "one":
                r = run_problem_one(n, var, args.precision, args.tol, args.maxit, not args.no_warmup, args.order,
                                    args.amg)
            else:
                r = run_problem_two(n, args.steps, var, args.precision, args.tol, args.maxit, args.delta_min,
                                    args.order, args.amg)
            print(json.dumps(r), flush=True)



def run_problem_two(n: int, steps: int, variant: str = "svn", precision: str = "fp64", tol: float = 1e-4,
                    maxit: int = 200, delta_min: float = 2e-9, order: int = 1, amg: str = "sa") -> dict:
    """The paper's Problem II (Sec. 5.3) for `steps` half-hour steps: each step
    advances A and H explicitly with the previous velocity (Sec. 3), then solves
    the momentum step from the previous (v, pi) until the residual has dropped by
    `tol` relative to its value at that start (the paper's 10^4 reduction)."""
    w = inputs.problem_two(n, delta_min, order)
    ctx = vp.context_for(w)
    st = ctx._state
    v = torch.zeros(ctx.node_shape, dtype=torch.float64, device="cuda")
    pi = torch.zeros(ctx.pi_shape, dtype=torch.float64, device="cuda")
    zero = torch.zeros_like(v)
    A, H = st["A"].clone(), st["H"].clone()
    A2, H2 = torch.empty_like(A), torch.empty_like(H)
    no, ao, ko = vp.default_opts()
    no.variant = vp.VP_SVN if variant == "svn" else vp.VP_STDN
    ao.precision = PREC[precision]
    ao.kind = vp.VP_AMG_RS if amg == "rs" else vp.VP_AMG_SA
    its, kits, fails = [], [], 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        ctx.vp_advect(v, A, H, A2, H2)
        A, A2, H, H2 = A2, A, H2, H
        va = vp.to_device(inputs.problem_two_wind(order * n, (k + 1) * w.desc.dt).reshape(-1, 2))
        ctx.vp_set_state(H, A, va, st["v_ocean"], v)
        r_start, _ = ctx.vp_residual(v)
        r_zero, _ = ctx.vp_residual(zero)
        no.tol = tol * r_start / r_zero if r_zero > 0 else tol
        rc, info, _ = ctx.vp_newton_solve(v, pi, maxit, no, ao, ko, history=False)
        its.append(info.iterations)
        kits.append(info.krylov_iters)
        fails += int(rc != 0)
        if (k + 1) % 24 == 0:
            print(f"[problem_two] n={n} {variant} step {k + 1}/{steps}: newton {info.iterations} "
                  f"mean {sum(its) / len(its):.2f}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out = dict(problem="problem_two", n=n, order=order, amg=amg, dx_km=512.0 / n, steps=steps, variant=variant,
               precision=precision,
               delta_min=delta_min, tol=tol, mean_newton=sum(its) / len(its), max_newton=max(its),
               total_krylov=sum(kits), failed_steps=fails, seconds=dt, newton_per_step=its,
               A_mean=float(A.mean()), H_mean=float(H.mean()))
    ctx.close()
    return out


if __name__ == "__main__":
    main()
