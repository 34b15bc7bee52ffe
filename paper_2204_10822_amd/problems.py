"""The paper's single momentum solve, Problem I (Sec. 5.2), on the GPU path.

Runs the stress-velocity Newton method (svN) and the standard Newton method
(stdN) on Problem I at 1 km, 0.5 km and 0.25 km (512^2, 1024^2, 2048^2 cells) with
the paper's stopping rule, a 10^4 reduction of the nonlinear residual, and a cap
of 200 Newton iterations, and prints one JSON line per run: Newton and Krylov
iterations, the reached reduction and the wall time of the solve.

    python -m paper_2204_10822_amd.problems --n 512,1024,2048 --variants svn,std
"""
from __future__ import annotations

import argparse
import json
import time

import torch

from . import inputs, vp

PREC = {"fp64": vp.VP_PREC_FP64, "fp32": vp.VP_PREC_FP32, "bf16": vp.VP_PREC_FP32_BF16COARSE,
        "fp16": vp.VP_PREC_FP16_BF16COARSE}


def run_problem_one(n: int, variant: str, precision: str = "fp64", tol: float = 1e-4, maxit: int = 200,
                    warmup: bool = True) -> dict:
    w = inputs.problem_one(n)
    ctx = vp.context_for(w)
    nn = (n + 1) ** 2
    v = torch.zeros(nn, 2, dtype=torch.float64, device="cuda")
    pi = torch.zeros(4, 3, n, n, dtype=torch.float64, device="cuda")
    no, ao, ko = vp.default_opts()
    no.variant = vp.VP_SVN if variant == "svn" else vp.VP_STDN
    no.tol = tol
    ao.precision = PREC[precision]

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
    return dict(problem="problem_one", n=n, dx_km=512.0 / n, variant=variant, precision=precision,
                tol=tol, maxit=maxit, rc=rc, converged=info.rel_resid <= tol,
                newton_its=info.iterations, krylov_its=info.krylov_iters, rel_resid=info.rel_resid,
                seconds=dt, history=[float(h) for h in hist])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", default="512,1024,2048")
    ap.add_argument("--variants", default="svn,std")
    ap.add_argument("--precision", default="fp64", choices=sorted(PREC))
    ap.add_argument("--tol", type=float, default=1e-4)
    ap.add_argument("--maxit", type=int, default=200)
    ap.add_argument("--no-warmup", action="store_true")
    args = ap.parse_args()
    torch.cuda.set_device(0)
    for n in [int(x) for x in args.n.split(",") if x]:
        for var in [x for x in args.variants.split(",") if x]:
            r = run_problem_one(n, var, args.precision, args.tol, args.maxit, not args.no_warmup)
            print(json.dumps(r), flush=True)


if __name__ == "__main__":
    main()
