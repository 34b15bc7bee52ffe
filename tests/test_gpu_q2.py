"""Q2 (biquadratic) velocity elements through the C ABI against the oracle's Q2
discretisation (Sec. 5): residual and energy, the svN and stdN operators (block
25-point stencil), the dual update, the AMG's first coarse level (tentative
Galerkin product of the Q2 operator), Krylov solves and full Newton solves."""
import numpy as np
import pytest
import scipy.sparse as sp
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


def _case(vp, nx, ny, seed, **kw):
    w = inputs.synthetic(nx, seed, ny=ny, Ly=512e3 * ny / nx, order=2, **kw)
    rng = np.random.default_rng(seed)
    w.v_prev = 0.05 * rng.standard_normal(w.v_prev.shape)
    print(f"[q2 case] nx={nx} ny={ny} seed={seed}", flush=True)
    prob = O.problem_from_workload(w)
    ctx = vp.context_for(w)
    return w, prob, ctx


def _rand_v(prob, seed, scale=0.1):
    rng = np.random.default_rng(seed)
    v = scale * rng.standard_normal(2 * prob.mesh.nnode)
    v[~prob.mesh.free_dof] = 0.0
    return v


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64).cuda()


def _host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def _relerr(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300)


# stored offsets of the symmetric 25-point stencil: self, (1,0), (2,0), (-2..2, 1), (-2..2, 2)
OFFS = [(0, 0), (1, 0), (2, 0)] + [(ox, 1) for ox in range(-2, 3)] + [(ox, 2) for ox in range(-2, 3)]


def _q2_matrix(vp, ctx, nxn, nyn):
    nn = nxn * nyn
    blocks = torch.zeros(52, nn, dtype=torch.float64, device="cuda")
    ctx.vp_operator_export(blocks)
    Bk = _host(blocks).reshape(13, nn, 2, 2)
    jj, ii = np.divmod(np.arange(nn), nxn)
    rows, cols, vals = [], [], []
    for b, (di, dj) in enumerate(OFFS):
        ok = (ii + di >= 0) & (ii + di < nxn) & (jj + dj < nyn)
        n = np.nonzero(ok)[0]
        m = (jj[n] + dj) * nxn + ii[n] + di
        for r in range(2):
            for c in range(2):
                rows.append(2 * n + r); cols.append(2 * m + c); vals.append(Bk[b, n, r, c])
                if b > 0:
                    rows.append(2 * m + c); cols.append(2 * n + r); vals.append(Bk[b, n, r, c])
    K = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(2 * nn, 2 * nn)).tocsr()
    K.sum_duplicates()
    return K


SHAPES = [(4, 3, 1), (9, 7, 2), (16, 16, 3)]


@pytest.mark.parametrize("nx,ny,seed", SHAPES)
def test_q2_residual_energy_parity(vp, nx, ny, seed):
    w, prob, ctx = _case(vp, nx, ny, seed)
    v = _rand_v(prob, seed + 10)
    r = torch.zeros(prob.mesh.nnode, 2, dtype=torch.float64, device="cuda")
    rn, en = ctx.vp_residual(_dev(v.reshape(-1, 2)), r)
    R = prob.residual(v)
    E, _ = prob.energy(v)
    er = _relerr(_host(r), R)
    print(f"[q2 residual] rel err {er:.2e}  energy {en:.6e} vs {E:.6e}", flush=True)
    assert er < 1e-12
    assert rn == pytest.approx(np.linalg.norm(R), rel=1e-12)
    assert en == pytest.approx(E, rel=1e-11)


@pytest.mark.parametrize("variant", ["svn", "std"])
@pytest.mark.parametrize("nx,ny,seed", SHAPES)
def test_q2_operator_parity(vp, nx, ny, seed, variant):
    w, prob, ctx = _case(vp, nx, ny, seed)
    v = _rand_v(prob, seed + 20)
    rng = np.random.default_rng(seed + 30)
    pi = 0.6 * rng.standard_normal((9, 3, ny, nx))
    ctx.vp_newton_assemble(_dev(v.reshape(-1, 2)), _dev(pi),
                           vp.VP_SVN if variant == "svn" else vp.VP_STDN)
    K = _q2_matrix(vp, ctx, prob.mesh.nxn, prob.mesh.nyn)
    Kr = prob.jacobian_svn(v, pi) if variant == "svn" else prob.jacobian_std(v)
    err = spla.norm(K - Kr) / spla.norm(Kr)
    print(f"[q2 operator] {variant} rel err {err:.2e}", flush=True)
    assert err < 1e-12
    # the operator product matches the exported matrix
    x = rng.standard_normal(2 * prob.mesh.nnode)
    y = torch.zeros(prob.mesh.nnode, 2, dtype=torch.float64, device="cuda")
    ctx.vp_operator_apply(_dev(x.reshape(-1, 2)), y)
    assert _relerr(_host(y), Kr @ x) < 1e-12


@pytest.mark.parametrize("nx,ny,seed", SHAPES[:2])
def test_q2_pi_update_and_init_parity(vp, nx, ny, seed):
    w, prob, ctx = _case(vp, nx, ny, seed)
    v = _rand_v(prob, seed + 40)
    dv = _rand_v(prob, seed + 41)
    rng = np.random.default_rng(seed + 42)
    pi = 0.5 * rng.standard_normal((9, 3, ny, nx))
    pt = _dev(pi)
    ctx.vp_pi_update(_dev(v.reshape(-1, 2)), _dev(dv.reshape(-1, 2)), pt, 0.37)
    ref = pi + 0.37 * prob.pi_step(v, dv, pi)
    assert _relerr(_host(pt), ref) < 1e-12
    ctx.vp_pi_init(_dev(v.reshape(-1, 2)), pt)
    assert _relerr(_host(pt), prob.pi_consistent(v)) < 1e-12


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_q2_krylov_with_amg(vp, prec):
    """FCG on the Q2 svN system: the V-cycle smooths the finest level with the Q2
    operator, restricts with the tentative prolongator and continues on
    Ptent^T K2 Ptent; converges to the direct solution."""
    nx, ny, seed = 24, 20, 4
    w, prob, ctx = _case(vp, nx, ny, seed)
    v = O.newton_solve(prob, maxit=2).v
    pi = prob.pi_consistent(v)
    ctx.vp_newton_assemble(_dev(v.reshape(-1, 2)), _dev(pi), vp.VP_SVN)
    n, a, k = vp.default_opts()
    a.precision = prec
    ctx.vp_amg_setup(a)
    b = -prob.residual(v)
    x = torch.zeros(prob.mesh.nnode, 2, dtype=torch.float64, device="cuda")
    k.rtol, k.maxit = 1e-10, 400
    rc, info = ctx.vp_krylov_solve(_dev(b.reshape(-1, 2)), x, k)
    print(f"[q2 krylov] prec={prec} its={info.iters} rel={info.rel_resid:.2e}", flush=True)
    assert rc == 0
    xd = spla.spsolve(prob.jacobian_svn(v, pi).tocsc(), b)
    assert _relerr(_host(x), xd) < 1e-6
    assert info.iters < 120  # measured 80-87


def _stencil9(blocks, nxn, nyn, B):
    """CSR matrix of a symmetric block 9-point stencil (5 stored blocks: self, E, N, NE, NW)."""
    nn = nxn * nyn
    A = blocks.reshape(5, nn, B, B)
    jj, ii = np.divmod(np.arange(nn), nxn)
    rows, cols, vals = [], [], []
    for b, (di, dj) in enumerate([(0, 0), (1, 0), (0, 1), (1, 1), (-1, 1)]):
        ok = (ii + di >= 0) & (ii + di < nxn) & (jj + dj < nyn)
        n = np.nonzero(ok)[0]
        m = (jj[n] + dj) * nxn + ii[n] + di
        for r in range(B):
            for c in range(B):
                rows.append(B * n + r); cols.append(B * m + c); vals.append(A[b, n, r, c])
                if b > 0:
                    rows.append(B * m + c); cols.append(B * n + r); vals.append(A[b, n, r, c])
    M = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(B * nn, B * nn)).tocsr()
    M.sum_duplicates()
    return M


@pytest.mark.parametrize("nx,ny,seed", [(16, 16, 3), (23, 14, 4)])
def test_q2_first_coarse_level_is_tentative_galerkin(vp, nx, ny, seed):
    """Level 1 of the Q2 hierarchy is Ptent^T K2 Ptent: the exported prolongator has
    only its own-aggregate slot, and the exported level-1 operator equals the
    product formed here from it and the exported K2 (empty coarse dofs aside)."""
    w, prob, ctx = _case(vp, nx, ny, seed)
    v = _rand_v(prob, 8, 0.05)
    ctx.vp_newton_assemble(_dev(v.reshape(-1, 2)), _dev(prob.pi_consistent(v)), vp.VP_SVN)
    ctx.vp_amg_setup()
    levels = ctx.vp_amg_info()
    (nxn, nyn, B0), (cx, cy, B1) = levels[0], levels[1]
    assert (nxn, nyn, B0) == (2 * nx + 1, 2 * ny + 1, 2) and B1 == 3
    nn, ncn = nxn * nyn, cx * cy
    P = torch.zeros(12 * B0, nn, dtype=torch.float64, device="cuda")
    A1 = torch.zeros(5 * 9 * ncn, dtype=torch.float64, device="cuda")
    ctx.vp_amg_export(0, None, P)
    ctx.vp_amg_export(1, A1, None)
    Pm = _host(P).reshape(4, B0, 3, nn)
    assert np.all(Pm[1:] == 0.0)
    agg = lambda i, na: np.minimum(i // 3, na - 1)
    jj, ii = np.divmod(np.arange(nn), nxn)
    I = agg(jj, cy) * cx + agg(ii, cx)
    rows, cols, vals = [], [], []
    for r in range(B0):
        for c in range(3):
            rows.append(B0 * np.arange(nn) + r); cols.append(3 * I + c); vals.append(Pm[0, r, c])
    Pt = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(B0 * nn, 3 * ncn))
    K2 = _q2_matrix(vp, ctx, nxn, nyn)
    G = (Pt.T @ K2 @ Pt).toarray()
    d = np.diag(G).copy()
    d[d == 0.0] = 1.0
    np.fill_diagonal(G, d)
    Ac = _stencil9(_host(A1), cx, cy, 3).toarray()
    err = np.linalg.norm(Ac - G) / np.linalg.norm(G)
    print(f"[q2 galerkin] {levels[:2]} rel err {err:.2e}", flush=True)
    assert err < 1e-13


def test_q2_rejects_scaled_16bit_vcycle(vp):
    """The Jacobi-scaled 16-bit finest level exists for Q1 only."""
    w, prob, ctx = _case(vp, 8, 8, 3)
    v = torch.zeros(prob.mesh.nnode, 2, dtype=torch.float64, device="cuda")
    pi = torch.zeros(9, 3, 8, 8, dtype=torch.float64, device="cuda")
    ctx.vp_pi_init(v, pi)
    ctx.vp_newton_assemble(v, pi, vp.VP_SVN)
    n, a, k = vp.default_opts()
    for prec in (3, 4, 5):
        a.precision = prec
        with pytest.raises(vp.VPError):
            ctx.vp_amg_setup(a)


@pytest.mark.parametrize("variant", ["svn", "std"])
def test_q2_newton_solve_parity(vp, variant):
    nx, ny, seed = 16, 14, 5
    w, prob, ctx = _case(vp, nx, ny, seed)
    ref = O.newton_solve(prob, variant=variant, tol=1e-8, maxit=200)
    assert ref.converged
    v = torch.zeros(prob.mesh.nnode, 2, dtype=torch.float64, device="cuda")
    pi = torch.zeros(9, 3, ny, nx, dtype=torch.float64, device="cuda")
    n, a, k = vp.default_opts()
    n.variant = vp.VP_SVN if variant == "svn" else vp.VP_STDN
    rc, info, hist = ctx.vp_newton_solve(v, pi, 200, n, a, k)
    err = _relerr(_host(v).ravel(), ref.v)
    print(f"[q2 newton] {variant} its {info.iterations} (oracle {ref.iterations}) krylov {info.krylov_iters} "
          f"rel {info.rel_resid:.2e} |v - v_oracle| {err:.2e}", flush=True)
    assert rc == 0 and info.rel_resid <= 1e-8
    assert err < 1e-6


def test_q2_advect_parity(vp):
    """Transport with Q2 velocity (Simpson face means) against the oracle."""
    from oracle import transport as T
    nx, ny = 21, 13
    w = inputs.synthetic(nx, 9, ny=ny, Ly=0.45 * 512e3, order=2)
    rng = np.random.default_rng(12)
    v = 0.3 * rng.standard_normal((2 * ny + 1, 2 * nx + 1, 2))
    v[0], v[-1], v[:, 0], v[:, -1] = 0.0, 0.0, 0.0, 0.0
    A = np.clip(w.A + 0.02 * rng.standard_normal(w.A.shape), 0.0, 1.0)
    ctx = vp.context_for(w)
    Ao = torch.empty(ny, nx, dtype=torch.float64, device="cuda")
    Ho = torch.empty(ny, nx, dtype=torch.float64, device="cuda")
    ctx.vp_advect(_dev(v.reshape(-1, 2)), _dev(A), _dev(w.H), Ao, Ho)
    Ar, Hr = T.advect(v.ravel(), A, w.H, nx, ny, w.desc.Lx, w.desc.Ly, w.desc.dt, order=2)
    ea = np.abs(_host(Ao) - Ar).max()
    eh = np.abs(_host(Ho) - Hr).max() / np.abs(Hr).max()
    print(f"[q2 advect] max |dA| {ea:.2e} max |dH|/max H {eh:.2e}", flush=True)
    assert ea < 1e-14 and eh < 1e-14
