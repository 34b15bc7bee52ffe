"""The library's inexact-Newton control against the oracle's: the inner tolerance
of every Newton step taken on the GPU (vp_newton_step, reported in
vp_newton_info.eta) is the oracle's Eisenstat-Walker choice (with its safeguard,
cap and floor) applied to the residual norms the GPU reports.  The two are
independent implementations (C++ host code in the library, Python in oracle/)."""
import numpy as np
import pytest

from oracle import vp_oracle as O
from paper_2204_10822_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def vp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2204_10822_amd import vp as _vp
    return _vp


@pytest.mark.parametrize("prec", [0, 1])
def test_forcing_terms_follow_the_oracle(vp, prec):
    w = inputs.synthetic(64, 5, (0.05, 1.5), (0.7, 1.0), 25.0, 2e-10)
    ctx = vp.context_for(w)
    v = torch.zeros(ctx.node_shape, dtype=torch.float64, device="cuda")
    pi = torch.zeros(ctx.pi_shape, dtype=torch.float64, device="cuda")
    no, ao, ko = vp.default_opts()
    ao.precision = prec
    no.tol = 1e-7
    rns, etas, r0 = [], [], None
    for _ in range(60):
        rc, info = ctx.vp_newton_step(v, pi, no, ao, ko)
        assert rc == 0
        rns.append(info.rnorm)
        etas.append(info.eta)
        r0 = info.rnorm0
        if info.rnorm_new <= no.tol * info.rnorm0:
            break
    ctx.close()
    print(f"[forcing] prec={prec} steps={len(rns)} etas {np.array(etas)}", flush=True)
    assert rns[-1] > 0 and len(rns) >= 4
    rn_prev, eta_prev, floored = None, no.eta_max, 0
    for rn, eta in zip(rns, etas):
        ref = O.eisenstat_walker(rn, rn_prev, eta_prev, no.tol * r0, no.eta_max)
        assert abs(eta - ref) <= 1e-14 * ref, (rn, eta, ref)
        floored += 0.5 * no.tol * r0 / rn >= ref * (1.0 - 1e-14)   # the floor (or the cap above it) decides
        rn_prev, eta_prev = rn, ref
    assert floored >= 1   # the floor against oversolving decides at least the last step
