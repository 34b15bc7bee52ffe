"""The learned warm start at the C ABI (vpnet_infer) and what the committed
trained network gains: the start is built from the context's step data by the
library's kernels, chosen by energy, and Newton always finishes the solve."""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def vp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2204_10822_amd import vp as _vp
    return _vp


@pytest.fixture(scope="module")
def ws(vp):
    from paper_2204_10822_amd import warmstart as W
    if not os.path.exists(W.WEIGHTS):
        pytest.skip("no trained weights committed")
    return W.WarmStart()


def _step2_state(vp, W, seed, n):
    """Context on the second step of a seeded sequence (v_prev = the first step's solution)."""
    w1 = W.sample_workload(seed, n)
    ctx = vp.Context(w1.desc)
    f = W.device_fields(w1)
    W.set_state(ctx, f)
    v = torch.zeros(ctx.node_shape, dtype=torch.float64, device="cuda")
    pi = torch.zeros(ctx.pi_shape, dtype=torch.float64, device="cuda")
    rc, _ = W.solve(ctx, v, pi, precision=vp.VP_PREC_FP32)
    assert rc == 0
    f2 = W.device_fields(W.sample_workload(seed, n, t=w1.desc.dt))
    f2["v_prev"] = v.clone()
    W.set_state(ctx, f2)
    return ctx, f2


def test_infer_candidates(vp, ws):
    from paper_2204_10822_amd import warmstart as W
    n = 256
    ctx, f = _step2_state(vp, W, 90100, n)
    v0 = torch.empty(ctx.node_shape, dtype=torch.float64, device="cuda")
    p0 = torch.empty(ctx.pi_shape, dtype=torch.float64, device="cuda")
    # zero
    v0.fill_(1.0); p0.fill_(1.0)
    assert ws.start(ctx, v0, p0, ("zero",)) == "zero"
    assert torch.count_nonzero(v0) == 0 and torch.count_nonzero(p0) == 0
    # previous: v_prev with pi = tau/Delta
    assert ws.start(ctx, v0, p0, ("previous",)) == "previous"
    pref = torch.empty_like(p0)
    ctx.vp_pi_init(f["v_prev"], pref)
    assert torch.equal(v0, f["v_prev"]) and torch.equal(p0, pref)
    # learned: the same kernels as features -> forward -> guess (v_prev + change)
    assert ws.start(ctx, v0, p0, ("learned",)) == "learned"
    feat = torch.zeros(n * n * 8, dtype=torch.float32, device="cuda")
    out = torch.zeros(n * n * 5, dtype=torch.float32, device="cuda")
    vp.vpnet_features(n, n, 1, f["H"], f["A"], f["v_air"], f["v_ocean"], f["v_prev"], feat)
    ws.net.vpnet_forward(feat, out)
    vm = torch.empty_like(v0)
    pm = torch.empty_like(p0)
    vp.vpnet_guess(n, n, out, n, n, vm, pm, v_prev=f["v_prev"])
    torch.cuda.synchronize()
    assert torch.equal(v0, vm) and torch.equal(p0, pm)
    # all three: the lowest energy wins
    energies = {}
    for name, vv in (("learned", vm), ("previous", f["v_prev"]), ("zero", torch.zeros_like(v0))):
        energies[name] = ctx.vp_residual(vv)[1]
    chosen = ws.start(ctx, v0, p0, ("learned", "previous", "zero"))
    print(f"[infer] energies {energies} chosen {chosen}", flush=True)
    assert chosen == min(energies, key=energies.get)


def test_infer_pools_larger_meshes_and_rejects_others(vp, ws):
    """On a mesh f times the network's grid (f > 1) the inputs are pooled and the
    proposed change is damped by VPNET_POOLED_SCALE with pi consistent with the
    damped velocity; beyond VPNET_MAX_POOL the learned start is no candidate; a
    mesh that is not a multiple of the grid is rejected."""
    from paper_2204_10822_amd import inputs, warmstart as W
    n, f = 512, 2
    w = W.sample_workload(90101, n)
    ctx = vp.context_for(w)
    st = ctx._state
    v0 = torch.empty(ctx.node_shape, dtype=torch.float64, device="cuda")
    p0 = torch.empty(ctx.pi_shape, dtype=torch.float64, device="cuda")
    assert ws.start(ctx, v0, p0, ("learned",)) == "learned"
    assert bool(torch.isfinite(v0).all()) and bool(torch.isfinite(p0).all())
    R = W.NET_RES
    feat = torch.zeros(R * R * 8, dtype=torch.float32, device="cuda")
    out = torch.zeros(R * R * 5, dtype=torch.float32, device="cuda")
    vp.vpnet_features(n, n, f, st["H"], st["A"], st["v_air"], st["v_ocean"], st["v_prev"], feat)
    ws.net.vpnet_forward(feat, out)
    vm = torch.empty_like(v0)
    pm = torch.empty_like(p0)
    vp.vpnet_guess(n, n, out, R, R, vm, pm, v_prev=st["v_prev"])
    s_ = vp.VPNET_POOLED_SCALE
    vexp = (1.0 - s_) * st["v_prev"] + s_ * vm
    pexp = torch.empty_like(p0)
    ctx.vp_pi_init(v0, pexp)
    torch.cuda.synchronize()
    err = float((v0 - vexp).abs().max() / vm.abs().max())
    print(f"[infer pooled] f={f} damped start vs scale*proposal: {err:.2e}", flush=True)
    assert err < 1e-14
    assert float((v0 - vm).abs().max()) > 0.1 * float(vm.abs().max())   # really damped
    assert torch.equal(p0, pexp)
    # more than VPNET_MAX_POOL times the grid per side (a 16^2 network on 144^2 cells)
    small = vp.Net(1, 16, 16)
    small.vpnet_set_params(torch.full((small.nparam,), 0.01, dtype=torch.float32, device="cuda"))
    fine = vp.context_for(inputs.synthetic(16 * (vp.VPNET_MAX_POOL + 1), 5))
    vf = torch.full(fine.node_shape, 7.0, dtype=torch.float64, device="cuda")
    pf = torch.full(fine.pi_shape, 7.0, dtype=torch.float64, device="cuda")
    assert small.vpnet_infer(fine, ("learned", "zero"), vf, pf) == "zero"
    assert torch.count_nonzero(vf) == 0 and torch.count_nonzero(pf) == 0
    with pytest.raises(vp.VPError) as e:
        small.vpnet_infer(fine, ("learned",), vf, pf)
    assert e.value.code == vp.VP_EINVAL
    bad = vp.context_for(inputs.synthetic(300, 5))
    vb = torch.empty(bad.node_shape, dtype=torch.float64, device="cuda")
    pb = torch.empty(bad.pi_shape, dtype=torch.float64, device="cuda")
    with pytest.raises(vp.VPError) as e:
        ws.start(bad, vb, pb, ("learned", "zero"))
    assert e.value.code == vp.VP_EINVAL


def test_learned_start_saves_newton_iterations(vp, ws):
    """Eight held-out 256^2 seeds (the training seeds are 10000-11999): from rest the
    learned start needs fewer Newton iterations on average than the zero start, and
    every solve reaches the same velocity (the minimiser is unique).  The second step
    of each sequence is reported against the previous-step start."""
    from paper_2204_10822_amd import warmstart as W
    rows = W.evaluate(ws, range(90000, 90008), 256, precision=vp.VP_PREC_FP32)
    s = W.summarize(rows)
    print("[learned] step 1: " + ", ".join(f"{k} {d['mean_newton']:.2f}" for k, d in s["step1"].items()), flush=True)
    print("[learned] step 2: " + ", ".join(f"{k} {d['mean_newton']:.2f}" for k, d in s["step2"].items())
          + f" (learned chosen {s['step2']['learned']['learned_used']} of 8)", flush=True)
    for r in rows:
        for m in W.MODES[r["step"]]:
            assert r[m]["rc"] == 0
            assert r[m]["rel_diff_vs_zero"] < 1e-6
    assert s["step1"]["learned"]["mean_newton"] < s["step1"]["zero"]["mean_newton"]
