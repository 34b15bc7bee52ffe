"""Write the oracle's converged velocities used as parity goldens (test infrastructure).

Calls only the CPU oracle (oracle/vp_oracle.py) and the seeded input generators;
nothing here touches the HIP library.  Each golden is the oracle's stress-velocity
Newton solve (Sec. 4.2, 5.1) from v = 0 with direct inner solves, run to a
nonlinear residual of 1e-10 relative to ||R(0)|| so that its own error sits well
below the 1e-6 the tests allow.  The discrete problem has a unique minimiser
(the strictly convex energy of eq. energy), so any correct solver reaches it.

    python tests/golden/make_goldens.py [name ...]      # default: all

Output: tests/golden/<name>.npz with v [(n+1)^2 * 2] float64 and the solve's
iteration count, final relative residual and ||R(0)||; for a step sequence the
last step's v and every step's iteration count and residual.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import vp_oracle as O            # noqa: E402
from paper_2204_10822_amd import inputs      # noqa: E402

TOL = 1e-10


def workloads():
    """name -> workload.  medium_512: the 512^2 multi-step recipe at its first step
    (seed 2, wind 15 m/s); problem_one_512: the paper's Problem I at 1 km (Sec. 5.2);
    sharp_512: the 2048^2 benchmark recipe (wind 25 m/s, H in [0.05, 1.5] m,
    Delta_min = 2e-10) on a 512^2 mesh."""
    return {"medium_512": lambda: inputs.medium_steps(512),
            "problem_one_512": lambda: inputs.problem_one(512),
            "sharp_512": lambda: inputs.synthetic(512, 3, (0.05, 1.5), (0.7, 1.0), 25.0, 2e-10,
                                                  name="vp_sharp_512")}


SEQUENCES = {"medium_512_steps10": (lambda: inputs.medium_steps(512), 10)}


def make_sequence(name: str) -> None:
    """The oracle's velocity after a sequence of implicit steps (Sec. 3): step k's
    previous velocity is the oracle's own step k-1 solution, each solve starting
    from it; A and H stay fixed, the wind's vortices drift."""
    mk, steps = SEQUENCES[name]
    w0 = mk()
    v = np.zeros(w0.v_prev.size)
    its, rels = [], []
    t0 = time.perf_counter()
    for k in range(1, steps + 1):
        prob = O.problem_from_workload(inputs.sequence_step(w0, k, v))
        res = O.newton_solve(prob, v0=v, tol=TOL, maxit=200, inner="direct")
        rel = res.history[-1]["rel"]
        print(f"[golden] {name} step {k}: converged={res.converged} its={res.iterations} rel={rel:.3e} "
              f"({time.perf_counter() - t0:.0f} s)", flush=True)
        if not res.converged:
            raise SystemExit(f"{name} step {k}: oracle did not converge ({res.status})")
        v = res.v
        its.append(res.iterations)
        rels.append(rel)
    np.savez_compressed(os.path.join(HERE, f"{name}.npz"), v=v, iterations=np.array(its),
                        rel_resid=np.array(rels), steps=steps, tol=TOL)


def make(name: str) -> None:
    if name in SEQUENCES:
        return make_sequence(name)
    w = workloads()[name]()
    prob = O.problem_from_workload(w)
    t0 = time.perf_counter()
    res = O.newton_solve(prob, tol=TOL, maxit=200, inner="direct")
    dt = time.perf_counter() - t0
    r0 = np.linalg.norm(prob.residual(np.zeros_like(res.v)))
    rel = res.history[-1]["rel"]
    print(f"[golden] {name}: converged={res.converged} its={res.iterations} rel={rel:.3e} "
          f"({dt:.0f} s)", flush=True)
    if not res.converged:
        raise SystemExit(f"{name}: oracle did not converge ({res.status})")
    np.savez_compressed(os.path.join(HERE, f"{name}.npz"), v=res.v, iterations=res.iterations,
                        rel_resid=rel, rnorm0=r0, tol=TOL)


if __name__ == "__main__":
    for nm in sys.argv[1:] or list(workloads()) + list(SEQUENCES):
        make(nm)
