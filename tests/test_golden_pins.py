"""The stored oracle goldens (tests/golden/*.npz, written by make_goldens.py from
the CPU oracle alone) still solve the oracle's discrete equations for today's
seeded inputs: the oracle's residual at each stored velocity is at the stored
level (<= 1e-10 of ||R(0)||).  This ties the files to the oracle and the input
generators, so a drift in either fails here rather than in the GPU tests."""
import os

import numpy as np
import pytest

from oracle import vp_oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = os.path.join(HERE, "golden")


def _load(name):
    import importlib.util
    spec = importlib.util.spec_from_file_location("make_goldens", os.path.join(GOLD, "make_goldens.py"))
    mg = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mg)
    return mg.workloads()[name](), np.load(os.path.join(GOLD, f"{name}.npz"), allow_pickle=False)


@pytest.mark.parametrize("name", ["medium_512", "problem_one_512", "sharp_512"])
def test_golden_solves_the_oracle_equations(name):
    w, g = _load(name)
    prob = O.problem_from_workload(w)
    v = g["v"]
    assert v.shape == (2 * prob.mesh.nnode,)
    assert np.all(v[~prob.mesh.free_dof] == 0.0)
    r0 = np.linalg.norm(prob.residual(np.zeros_like(v)))
    rel = np.linalg.norm(prob.residual(v)) / r0
    print(f"[golden] {name}: oracle |R(v)|/|R(0)| = {rel:.3e} (stored {float(g['rel_resid']):.3e})")
    assert rel <= 1e-10
    assert r0 == pytest.approx(float(g["rnorm0"]), rel=1e-12)
