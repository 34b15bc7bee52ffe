"""Oracle parity at scale: GPU Newton solves on 512^2 meshes (526k unknowns)
against the CPU oracle's converged velocities (tests/golden, written by the
oracle alone to 1e-10), for the plain FP64 path, the FP32 V-cycle, the FP32 +
BF16-coarse mixed mode and the mixed mode from the learned start: each must
reach 1e-6 relative l2 at a nonlinear residual of 1e-8 of ||R(0)||."""
import importlib.util
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def vp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2204_10822_amd import vp as _vp
    return _vp


def _golden(name):
    spec = importlib.util.spec_from_file_location("make_goldens", os.path.join(GOLD, "make_goldens.py"))
    mg = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mg)
    return mg.workloads()[name](), np.load(os.path.join(GOLD, f"{name}.npz"), allow_pickle=False)["v"]


@pytest.mark.parametrize("name", ["medium_512", "problem_one_512", "sharp_512"])
@pytest.mark.parametrize("path", ["fp64", "fp32", "bf16", "bf16+learned"])
def test_newton_matches_oracle_golden(vp, name, path):
    w, vg = _golden(name)
    prec = {"fp64": vp.VP_PREC_FP64, "fp32": vp.VP_PREC_FP32}.get(path, vp.VP_PREC_FP32_BF16COARSE)
    print(f"[scale] {name} {path}", flush=True)
    ctx = vp.context_for(w)
    n = w.desc.nx
    v = torch.zeros(ctx.node_shape, dtype=torch.float64, device="cuda")
    pi = torch.zeros(ctx.pi_shape, dtype=torch.float64, device="cuda")
    no, ao, ko = vp.default_opts()
    ao.precision = prec
    start = "zero"
    if path.endswith("learned"):
        from paper_2204_10822_amd import warmstart as W
        if not os.path.exists(W.WEIGHTS):
            pytest.skip("no trained weights committed")
        rc, info, start = W.solve_with_fallback(ctx, W.WarmStart(), v, pi, ("learned", "zero"), no, ao, ko)
    else:
        rc, info, _ = ctx.vp_newton_solve(v, pi, 200, no, ao, ko, history=False)
    err = np.linalg.norm(v.cpu().numpy().ravel() - vg) / np.linalg.norm(vg)
    print(f"[scale] {name} {path}: rc={rc} start={start} newton={info.iterations} krylov={info.krylov_iters} "
          f"rel_resid={info.rel_resid:.2e} err_vs_oracle={err:.2e}", flush=True)
    assert rc == 0 and info.rel_resid <= 1e-8
    assert err < 1e-6
