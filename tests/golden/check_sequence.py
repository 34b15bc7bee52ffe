"""Oracle check of the last step of a GPU step sequence (test infrastructure).

    python tests/golden/check_sequence.py FILE.npz

FILE.npz is written by `python -m paper_2204_10822_amd.sequences c5 --save FILE`:
the last velocity of each path and the one before it.  For each path this
evaluates the CPU oracle's residual (eq. A - eq. F, Sec. 3) of the last step at
that path's last velocity, with the path's own previous velocity as v^n and the
drifted wind of that step: ||R(v)|| / ||R(0)||.  It checks a property of the
GPU result (it solves the oracle's discrete equations for the state it was
handed); it stores nothing.  Prints one JSON line.
"""
from __future__ import annotations

import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import vp_oracle as O            # noqa: E402
from paper_2204_10822_amd import inputs      # noqa: E402


def main(path):
    f = np.load(path, allow_pickle=False)
    n, steps = int(f["n"]), int(f["steps"])
    w0 = inputs.long_run(n)
    out = {}
    for name in ("fp64", "mixed"):
        prob = O.problem_from_workload(inputs.sequence_step(w0, steps, f[f"{name}_v_before"]))
        v = f[f"{name}_v"]
        rel = np.linalg.norm(prob.residual(v)) / np.linalg.norm(prob.residual(np.zeros_like(v)))
        out[f"{name}_oracle_rel_resid"] = float(rel)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main(sys.argv[1])
