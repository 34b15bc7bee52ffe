"""The allocation-free Krylov entry point (vp_krylov_solve_noalloc, workspace in a
static device array) against vp_krylov_solve with flexible CG: the same kernels on
the same data, so the iterates agree bitwise; both solve the oracle's operator.
Two calls in a row, the second on a smaller mesh (the static array keeps the
first call's contents)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

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


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64).cuda()


def _solve_pair(vp, nx, ny, seed, prec):
    w = inputs.synthetic(nx, seed, ny=ny, Ly=512e3 * ny / nx)
    print(f"[no-alloc] nx={nx} ny={ny} seed={seed} prec={prec}", flush=True)
    prob = O.problem_from_workload(w)
    ctx = vp.context_for(w)
    v = O.newton_solve(prob, maxit=2).v
    pi = prob.pi_consistent(v)
    ctx.vp_newton_assemble(_dev(v.reshape(-1, 2)), _dev(pi), vp.VP_SVN)
    _, a, k = vp.default_opts()
    a.precision = prec
    ctx.vp_amg_setup(a)
    b = _dev((-prob.residual(v)).reshape(-1, 2))
    k.method, k.rtol, k.maxit = vp.VP_KRYLOV_FCG, 1e-10, 400
    x_ref = torch.zeros_like(b)
    rc0, i0 = ctx.vp_krylov_solve(b, x_ref, k)
    x_na = torch.full_like(b, 0.0)
    rc1, i1 = ctx.vp_krylov_solve_noalloc(b, x_na, k)
    torch.cuda.synchronize()
    print(f"[no-alloc] its {i0.iters}/{i1.iters} rel {i0.rel_resid:.3e}/{i1.rel_resid:.3e}", flush=True)
    assert rc0 == rc1 == 0
    assert i0.iters == i1.iters and i0.rel_resid == i1.rel_resid
    xr, xn = x_ref.cpu().numpy().ravel(), x_na.cpu().numpy().ravel()
    assert np.array_equal(xr, xn)
    xd = spla.spsolve(prob.jacobian_svn(v, pi).tocsc(), -prob.residual(v))
    assert np.linalg.norm(xn - xd) / np.linalg.norm(xd) < 1e-6
    return ctx


def test_noalloc_krylov_matches_allocating_solve(vp):
    _solve_pair(vp, 96, 80, 21, vp.VP_PREC_FP32)
    _solve_pair(vp, 40, 33, 22, vp.VP_PREC_FP64)


def test_noalloc_krylov_errors(vp):
    w = inputs.synthetic(24, 23, ny=20, Ly=512e3 * 20 / 24)
    ctx = vp.context_for(w)
    b = torch.ones(ctx.node_shape, dtype=torch.float64, device="cuda")
    x = torch.zeros_like(b)
    _, _, k = vp.default_opts()
    k.method = vp.VP_KRYLOV_FCG
    with pytest.raises(vp.VPError) as e:
        ctx.vp_krylov_solve_noalloc(b, x, k)       # no operator yet
    assert e.value.code == vp.VP_ESTATE
    k.method = vp.VP_KRYLOV_FGMRES
    with pytest.raises(vp.VPError) as e:
        ctx.vp_krylov_solve_noalloc(b, x, k)
    assert e.value.code == vp.VP_EINVAL
    big = vp.Context(inputs.ProblemDesc(nx=1100, ny=1100))   # 2,424,402 dofs
    bb = torch.zeros(big.node_shape, dtype=torch.float64, device="cuda")
    k.method = vp.VP_KRYLOV_FCG
    with pytest.raises(vp.VPError) as e:
        big.vp_krylov_solve_noalloc(bb, bb.clone(), k)
    assert e.value.code == vp.VP_EINVAL and "too large" in str(e.value)
