"""Classical (Ruge-Stueben) AMG with the paper's settings (Sec. 5.4) on the GPU,
through the C ABI, against the classical-AMG oracle (oracle/rs_amg.py).

The coarsening and the colouring are not unique (the GPU takes the first pass
in parallel rounds, the oracle sequentially), so the GPU's splitting and
colouring are checked for validity and compared in size with the oracle's, and
everything they determine (interpolation, Galerkin operators, the V-cycle) is
rebuilt by the oracle from them and compared entry by entry."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import rs_amg as R
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


def _host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _relerr(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300)


def _case(vp, nx, ny, seed, order=1):
    w = inputs.synthetic(nx, seed, ny=ny, Ly=512e3 * ny / nx, order=order)
    rng = np.random.default_rng(seed)
    w.v_prev = 0.05 * rng.standard_normal(w.v_prev.shape)
    print(f"[rs case] nx={nx} ny={ny} seed={seed} order={order}", flush=True)
    prob = O.problem_from_workload(w)
    ctx = vp.context_for(w)
    v = O.newton_solve(prob, maxit=2).v
    pi = prob.pi_consistent(v)
    ctx.vp_newton_assemble(_dev(v.reshape(-1, 2)), _dev(pi), vp.VP_SVN)
    return w, prob, ctx, v, pi


def _rs_opts(vp, max_coarse=40):
    n, a, k = vp.default_opts()
    a.kind = vp.VP_AMG_RS
    a.max_coarse = max_coarse
    return n, a, k


def _csr(d, n, m=None):
    return sp.csr_matrix((_host(d[2]), _host(d[1]), _host(d[0])), shape=(n, m if m is not None else n))


def _export(ctx):
    levels = []
    nl = len(ctx.vp_amg_info())
    for l in range(nl):
        e = ctx.vp_amg_rs_export(l)
        n, nc = e["n"], e["nc"]
        lev = dict(n=n, nc=nc, ncol=e["ncol"], A=_csr((e["A_ptr"], e["A_col"], e["A_val"]), n))
        if nc > 0:
            lev.update(cf=_host(e["cf"]).astype(np.int64), colour=_host(e["colour"]).astype(np.int64),
                       P=_csr((e["P_ptr"], e["P_col"], e["P_val"]), n, nc))
        levels.append(lev)
    return levels


def _max_rel(A, B):
    D = (sp.csr_matrix(A) - sp.csr_matrix(B)).tocoo()
    scale = abs(sp.csr_matrix(B)).max()
    return (abs(D.data).max() if D.nnz else 0.0) / scale


SHAPES = [(12, 9, 1), (23, 17, 2), (40, 40, 3)]


@pytest.mark.parametrize("nx,ny,seed", SHAPES)
def test_rs_hierarchy_parity(vp, nx, ny, seed):
    w, prob, ctx, v, pi = _case(vp, nx, ny, seed)
    n, a, k = _rs_opts(vp)
    ctx.vp_amg_setup(a)
    levels = _export(ctx)
    print(f"[rs levels] {[(L['n'], L['A'].nnz, L.get('ncol')) for L in levels]}", flush=True)
    assert len(levels) >= 3
    # level 0 is the assembled operator with the vectors' dof numbering
    K = prob.jacobian_svn(v, pi).tocsr()
    K.eliminate_zeros()
    assert _max_rel(levels[0]["A"], K) < 1e-12  # GPU vs oracle assembly rounding
    for l, L in enumerate(levels[:-1]):
        A = L["A"]
        S = R.strength(A, theta=0.5, max_row_sum=0.9)
        cf = L["cf"]
        assert set(np.unique(cf)) <= {0, 1}
        assert L["nc"] == int(cf.sum())
        # the splitting's coarse count is close to the sequential first pass's
        cf_seq = R.rs_first_pass(S)
        assert abs(int(cf.sum()) - int(cf_seq.sum())) <= 0.25 * cf_seq.sum() + 2
        # F points with strong couplings but no strong C point: no more than sequentially
        def orphans(c):
            cnt = 0
            for i in np.nonzero(c == 0)[0]:
                js = S.indices[S.indptr[i]:S.indptr[i + 1]]
                cnt += int(js.size > 0 and not np.any(c[js] == 1))
            return cnt
        assert orphans(cf) <= orphans(cf_seq) + 0.02 * A.shape[0] + 2
        # interpolation and Galerkin operator rebuilt from the GPU's splitting
        P = R.interpolation(A, S, cf)
        assert _max_rel(L["P"], P) < 1e-13
        Ac = R.galerkin(A, L["P"])
        assert _max_rel(levels[l + 1]["A"], Ac) < 1e-13
        # a valid colouring of A's graph
        assert R.is_valid_colouring(A, L["colour"])
        assert L["ncol"] == int(L["colour"].max()) + 1


@pytest.mark.parametrize("nx,ny,seed", SHAPES[1:])
def test_rs_vcycle_parity_and_determinism(vp, nx, ny, seed):
    w, prob, ctx, v, pi = _case(vp, nx, ny, seed)
    n, a, k = _rs_opts(vp)
    ctx.vp_amg_setup(a)
    levels = _export(ctx)
    H = R.RSHierarchy(levels[0]["A"], theta=0.5, max_row_sum=0.9, sweeps=3, max_coarse=40,
                      splittings=[L["cf"] for L in levels[:-1]], colourings=[L["colour"] for L in levels[:-1]])
    assert len(H.A) == len(levels)
    rng = np.random.default_rng(seed + 7)
    r = rng.standard_normal(levels[0]["n"])
    z = torch.zeros(levels[0]["n"] // 2, 2, dtype=torch.float64, device="cuda")
    ctx.vp_amg_apply(_dev(r.reshape(-1, 2)), z)
    zg = _host(z).ravel()
    zo = H.vcycle(r)
    err = _relerr(zg, zo)
    print(f"[rs vcycle] levels {len(levels)} rel err {err:.2e}", flush=True)
    assert err < 1e-11
    # a second setup on the same operator gives bitwise the same V-cycle
    ctx.vp_amg_setup(a)
    z2 = torch.zeros_like(z)
    ctx.vp_amg_apply(_dev(r.reshape(-1, 2)), z2)
    assert torch.equal(z, z2)
    # the V-cycle is symmetric (symmetric sweeps, R = P^T)
    u = rng.standard_normal(levels[0]["n"])
    zu = torch.zeros_like(z)
    ctx.vp_amg_apply(_dev(u.reshape(-1, 2)), zu)
    lhs, rhs = u @ zg, r @ _host(zu).ravel()
    assert abs(lhs - rhs) <= 1e-10 * abs(lhs)


@pytest.mark.parametrize("method", ["fcg", "fgmres"])
def test_rs_krylov_solution(vp, method):
    w, prob, ctx, v, pi = _case(vp, 40, 40, 4)
    n, a, k = _rs_opts(vp)
    ctx.vp_amg_setup(a)
    b = -prob.residual(v)
    x = torch.zeros(prob.mesh.nnode, 2, dtype=torch.float64, device="cuda")
    k.method = vp.VP_KRYLOV_FCG if method == "fcg" else vp.VP_KRYLOV_FGMRES
    k.rtol, k.maxit = 1e-10, 300
    rc, info = ctx.vp_krylov_solve(_dev(b.reshape(-1, 2)), x, k)
    print(f"[rs krylov] {method} its={info.iters} rel={info.rel_resid:.2e}", flush=True)
    assert rc == 0
    xd = spla.spsolve(prob.jacobian_svn(v, pi).tocsc(), b)
    assert _relerr(_host(x), xd) < 1e-6
    assert info.iters < 100


def test_rs_newton_solve_parity(vp):
    w = inputs.synthetic(32, 5)
    prob = O.problem_from_workload(w)
    ref = O.newton_solve(prob, tol=1e-8, maxit=100)
    assert ref.converged
    ctx = vp.context_for(w)
    v = torch.zeros(prob.mesh.nnode, 2, dtype=torch.float64, device="cuda")
    pi = torch.zeros(4, 3, 32, 32, dtype=torch.float64, device="cuda")
    n, a, k = _rs_opts(vp)
    rc, info, hist = ctx.vp_newton_solve(v, pi, 100, n, a, k)
    err = _relerr(_host(v).ravel(), ref.v)
    print(f"[rs newton] its {info.iterations} (oracle {ref.iterations}) krylov {info.krylov_iters} "
          f"rel {info.rel_resid:.2e} |v - v_oracle| {err:.2e}", flush=True)
    assert rc == 0 and info.rel_resid <= 1e-8
    assert err < 1e-6


def test_rs_q2_operator(vp):
    """Classical AMG works on the Q2 operator directly (25-point stencil to CSR)."""
    w, prob, ctx, v, pi = _case(vp, 10, 8, 6, order=2)
    n, a, k = _rs_opts(vp)
    ctx.vp_amg_setup(a)
    levels = _export(ctx)
    K = prob.jacobian_svn(v, pi).tocsr()
    K.eliminate_zeros()
    assert _max_rel(levels[0]["A"], K) < 1e-12  # GPU vs oracle assembly rounding
    b = -prob.residual(v)
    x = torch.zeros(prob.mesh.nnode, 2, dtype=torch.float64, device="cuda")
    k.rtol, k.maxit = 1e-10, 300
    rc, info = ctx.vp_krylov_solve(_dev(b.reshape(-1, 2)), x, k)
    print(f"[rs q2 krylov] its={info.iters} rel={info.rel_resid:.2e}", flush=True)
    assert rc == 0
    xd = spla.spsolve(K.tocsc(), b)
    assert _relerr(_host(x), xd) < 1e-6


def test_rs_rejects_bad_options(vp):
    w, prob, ctx, v, pi = _case(vp, 8, 8, 7)
    n, a, k = _rs_opts(vp)
    for field, bad in (("precision", vp.VP_PREC_FP32), ("sweeps", 0), ("strong_threshold", 1.0),
                       ("max_row_sum", 0.0), ("kind", 7)):
        n, a, k = _rs_opts(vp)
        setattr(a, field, bad)
        with pytest.raises(vp.VPError):
            ctx.vp_amg_setup(a)
