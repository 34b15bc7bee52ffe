"""Parity of the HIP library (through its C ABI) with the CPU oracle.

FP64 kernels must agree with the oracle to 1e-12 in the normwise relative sense;
the Newton solve must reach the oracle's velocity to 1e-6 relative l2 at a
nonlinear residual of 1e-8 relative to ||R(0)||.
"""
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
    w = inputs.synthetic(nx, seed, ny=ny, Ly=512e3 * ny / nx, **kw)
    rng = np.random.default_rng(seed)
    w.v_prev = 0.05 * rng.standard_normal(w.v_prev.shape)
    print(f"[case] nx={nx} ny={ny} seed={seed}", flush=True)
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


def export_matrix(vp, ctx, nx, ny):
    """Build a scipy CSR matrix from the 5-block symmetric stencil storage."""
    nxn, nyn = nx + 1, ny + 1
    nn = nxn * nyn
    blocks = torch.zeros(20, nn, dtype=torch.float64, device="cuda")
    ctx.vp_operator_export(blocks)
    B = _host(blocks).reshape(5, nn, 2, 2).transpose(0, 2, 3, 1)   # [blk][r][c][node]
    jj, ii = np.divmod(np.arange(nn), nxn)
    offs = [(0, 0), (1, 0), (0, 1), (1, 1), (-1, 1)]
    rows, cols, vals = [], [], []
    for b, (di, dj) in enumerate(offs):
        ok = (ii + di >= 0) & (ii + di < nxn) & (jj + dj < nyn)
        n = np.nonzero(ok)[0]
        m = (jj[n] + dj) * nxn + ii[n] + di
        for r in range(2):
            for c in range(2):
                rows.append(2 * n + r); cols.append(2 * m + c); vals.append(B[b, r, c, n])
                if b > 0:
                    rows.append(2 * m + c); cols.append(2 * n + r); vals.append(B[b, r, c, n])
    K = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(2 * nn, 2 * nn)).tocsr()
    K.sum_duplicates()
    return K


SHAPES = [(8, 6, 1), (23, 17, 2), (64, 64, 3), (100, 37, 4)]


@pytest.mark.parametrize("nx,ny,seed", SHAPES)
def test_residual_energy_parity(vp, nx, ny, seed):
    w, prob, ctx = _case(vp, nx, ny, seed)
    for k, v in enumerate([np.zeros(2 * prob.mesh.nnode), _rand_v(prob, 10 + seed)]):
        r = torch.zeros(prob.mesh.nnode, 2, dtype=torch.float64, device="cuda")
        rn, en = ctx.vp_residual(_dev(v.reshape(-1, 2)), r)
        R = prob.residual(v)
        e, eabs = prob.energy(v)
        assert _relerr(_host(r), R) < 1e-12
        assert abs(rn - np.linalg.norm(R)) <= 1e-12 * np.linalg.norm(R)
        assert abs(en - e) <= 1e-12 * eabs


@pytest.mark.parametrize("nx,ny,seed", SHAPES)
@pytest.mark.parametrize("variant", ["svn", "std"])
def test_operator_parity(vp, nx, ny, seed, variant):
    w, prob, ctx = _case(vp, nx, ny, seed)
    v = _rand_v(prob, 20 + seed)
    rng = np.random.default_rng(seed)
    pi = 0.8 * rng.standard_normal((4, 3, ny, nx))       # includes |pi| > 1/sqrt2
    vt = _dev(v.reshape(-1, 2))
    ctx.vp_newton_assemble(vt, _dev(pi), vp.VP_SVN if variant == "svn" else vp.VP_STDN)
    Kg = export_matrix(vp, ctx, nx, ny)
    Ko = prob.jacobian_svn(v, pi) if variant == "svn" else prob.jacobian_std(v)
    assert spla.norm(Kg - Ko) <= 1e-12 * spla.norm(Ko)
    # operator apply (FP64 stencil SpMV)
    x = rng.standard_normal(2 * prob.mesh.nnode)
    y = torch.zeros(prob.mesh.nnode, 2, dtype=torch.float64, device="cuda")
    ctx.vp_operator_apply(_dev(x.reshape(-1, 2)), y)
    assert _relerr(_host(y), Ko @ x) < 1e-12


@pytest.mark.parametrize("nx,ny,seed", SHAPES[:3])
def test_pi_update_and_init_parity(vp, nx, ny, seed):
    w, prob, ctx = _case(vp, nx, ny, seed)
    v = _rand_v(prob, 30 + seed)
    dv = _rand_v(prob, 31 + seed, 0.02)
    rng = np.random.default_rng(seed)
    pi = 0.8 * rng.standard_normal((4, 3, ny, nx))
    pt = _dev(pi)
    ctx.vp_pi_update(_dev(v.reshape(-1, 2)), _dev(dv.reshape(-1, 2)), pt, 0.37)
    ref = pi + 0.37 * prob.pi_step(v, dv, pi)
    assert _relerr(_host(pt), ref) < 1e-12
    ctx.vp_pi_init(_dev(v.reshape(-1, 2)), pt)
    assert _relerr(_host(pt), prob.pi_consistent(v)) < 1e-12


@pytest.mark.parametrize("method", ["fgmres", "fcg"])
@pytest.mark.parametrize("prec", [0, 1, 2, 3, 4, 5, 6])
def test_krylov_solves_assembled_system(vp, method, prec):
    nx, ny, seed = 64, 48, 5
    w, prob, ctx = _case(vp, nx, ny, seed)
    v = O.newton_solve(prob, maxit=2).v
    pi = prob.pi_consistent(v)
    ctx.vp_newton_assemble(_dev(v.reshape(-1, 2)), _dev(pi), vp.VP_SVN)
    n, a, k = vp.default_opts()
    a.precision = prec
    ctx.vp_amg_setup(a)
    b = -prob.residual(v)
    x = torch.zeros(prob.mesh.nnode, 2, dtype=torch.float64, device="cuda")
    k.method = vp.VP_KRYLOV_FGMRES if method == "fgmres" else vp.VP_KRYLOV_FCG
    k.rtol, k.maxit = 1e-10, 400
    rc, info = ctx.vp_krylov_solve(_dev(b.reshape(-1, 2)), x, k)
    print(f"[krylov] {method} prec={prec} its={info.iters} rel={info.rel_resid:.2e}", flush=True)
    assert rc == 0
    K = prob.jacobian_svn(v, pi)
    xd = spla.spsolve(K.tocsc(), b)
    assert _relerr(_host(x), xd) < 1e-6
    assert info.iters < 120


def test_vcycle_is_symmetric_fp64(vp):
    """With pre- and post-smoothing by the same Chebyshev polynomial and an exact
    coarse solve the FP64 V-cycle is a symmetric operator."""
    nx, ny, seed = 40, 33, 6
    w, prob, ctx = _case(vp, nx, ny, seed)
    v = _rand_v(prob, 40)
    ctx.vp_newton_assemble(_dev(v.reshape(-1, 2)), _dev(prob.pi_consistent(v)), vp.VP_SVN)
    ctx.vp_amg_setup()
    rng = np.random.default_rng(7)
    x, y = rng.standard_normal((2, 2 * prob.mesh.nnode))
    x[~prob.mesh.free_dof] = 0.0
    y[~prob.mesh.free_dof] = 0.0
    zx = torch.zeros(prob.mesh.nnode, 2, dtype=torch.float64, device="cuda")
    zy = torch.zeros_like(zx)
    ctx.vp_amg_apply(_dev(x.reshape(-1, 2)), zx)
    ctx.vp_amg_apply(_dev(y.reshape(-1, 2)), zy)
    a, b = y @ _host(zx).ravel(), x @ _host(zy).ravel()
    assert abs(a - b) <= 1e-10 * max(abs(a), abs(b))
    assert a > 0


def test_determinism_bitwise(vp):
    """Two contexts on the same inputs give bitwise-equal residuals, energies and
    V-cycle outputs: reductions use fixed orders and no floating-point atomics."""
    nx, ny, seed = 64, 64, 8
    outs = []
    for _ in range(2):
        w, prob, ctx = _case(vp, nx, ny, seed)
        v = _rand_v(prob, 41)
        vt = _dev(v.reshape(-1, 2))
        r = torch.zeros(prob.mesh.nnode, 2, dtype=torch.float64, device="cuda")
        rn, en = ctx.vp_residual(vt, r)
        ctx.vp_newton_assemble(vt, _dev(prob.pi_consistent(v)), vp.VP_SVN)
        ctx.vp_amg_setup()
        z = torch.zeros_like(r)
        ctx.vp_amg_apply(r, z)
        outs.append((_host(r).copy(), rn, en, _host(z).copy()))
    assert np.array_equal(outs[0][0], outs[1][0]) and outs[0][1] == outs[1][1] and outs[0][2] == outs[1][2]
    assert np.array_equal(outs[0][3], outs[1][3])


@pytest.mark.parametrize("nx,ny,seed,variant", [(32, 32, 1, "svn"), (64, 64, 1, "svn"), (48, 40, 2, "std")])
def test_newton_solve_parity(vp, nx, ny, seed, variant):
    if (nx, ny, seed) == (64, 64, 1):
        w = inputs.small_step(64)
        prob = O.problem_from_workload(w)
        ctx = vp.context_for(w)
    else:
        w, prob, ctx = _case(vp, nx, ny, seed)
    ref = O.newton_solve(prob, variant=variant, tol=1e-8, maxit=200)
    assert ref.converged
    v = torch.zeros(prob.mesh.nnode, 2, dtype=torch.float64, device="cuda")
    pi = torch.zeros(4, 3, ny, nx, dtype=torch.float64, device="cuda")
    n, a, k = vp.default_opts()
    n.variant = vp.VP_SVN if variant == "svn" else vp.VP_STDN
    rc, info, hist = ctx.vp_newton_solve(v, pi, 200, n, a, k)
    print(f"[newton] {nx}x{ny} {variant}: gpu its={info.iterations} krylov={info.krylov_iters} "
          f"rel={info.rel_resid:.2e}; oracle its={ref.iterations}", flush=True)
    assert rc == 0
    assert info.rel_resid <= 1e-8
    assert _relerr(_host(v).ravel(), ref.v) < 1e-6
    if variant == "svn":
        assert abs(info.iterations - ref.iterations) <= 4
        assert _relerr(_host(pi), prob.pi_consistent(ref.v)) < 1e-4


def test_vcycle_reduced_precision_close_to_fp64(vp):
    """The FP32 V-cycle applies the same operator as the FP64 one up to FP32
    rounding; with BF16 coarse operators (Jacobi-scaled) the difference is of the
    order of BF16 rounding, with an FP16 finest level below that, and FP16 on
    every level of the order of FP16 rounding; FP16 finest smoothing with the
    post-correction residual and the coarse levels in FP32 lies between FP32 and
    FP16.  Fresh contexts give all the same spectral estimates."""
    nx, ny, seed = 64, 48, 5
    outs = {}
    for prec in (0, 1, 2, 3, 4, 5, 6):
        w, prob, ctx = _case(vp, nx, ny, seed)
        v = O.newton_solve(prob, maxit=2).v
        ctx.vp_newton_assemble(_dev(v.reshape(-1, 2)), _dev(prob.pi_consistent(v)), vp.VP_SVN)
        rng = np.random.default_rng(9)
        r = rng.standard_normal(2 * prob.mesh.nnode)
        r[~prob.mesh.free_dof] = 0.0
        n, a, k = vp.default_opts()
        a.precision = prec
        ctx.vp_amg_setup(a)
        z = torch.zeros(prob.mesh.nnode, 2, dtype=torch.float64, device="cuda")
        ctx.vp_amg_apply(_dev(r.reshape(-1, 2)), z)
        outs[prec] = _host(z).ravel()
    d32 = _relerr(outs[1], outs[0])
    dbf = _relerr(outs[2], outs[0])
    dba = _relerr(outs[3], outs[0])
    dh = _relerr(outs[4], outs[0])
    dha = _relerr(outs[5], outs[0])
    dhc = _relerr(outs[6], outs[0])
    print(f"[vcycle] fp32 vs fp64 {d32:.2e}  bf16-coarse vs fp64 {dbf:.2e}  bf16-all vs fp64 {dba:.2e}  "
          f"fp16-finest vs fp64 {dh:.2e}  fp16-all vs fp64 {dha:.2e}  fp16-finest-fp32-coarse vs fp64 {dhc:.2e}",
          flush=True)
    assert d32 < 1e-4
    assert dbf < 5e-2
    assert dba < 1e-1
    assert dh < 5e-2
    assert dha < 1e-2
    assert dhc < dha


def _stencil_matrix(blocks, nxn, nyn, B):
    """CSR matrix of a symmetric block 9-point stencil from the 5-block storage
    (blocks: [5][node][B][B] flattened, self, E, N, NE, NW)."""
    nn = nxn * nyn
    A = blocks.reshape(5, nn, B, B)
    jj, ii = np.divmod(np.arange(nn), nxn)
    offs = [(0, 0), (1, 0), (0, 1), (1, 1), (-1, 1)]
    rows, cols, vals = [], [], []
    for b, (di, dj) in enumerate(offs):
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


def _runs(n):
    """Aggregates along one axis: runs of 3 nodes, the last run takes 3..5."""
    na = n // 3
    own = np.minimum(np.arange(n) // 3, na - 1)
    other = np.full(n, -1)
    for a in range(na):
        first, last = 3 * a, (n - 1 if a == na - 1 else 3 * a + 2)
        if a > 0:
            other[first] = a - 1
        if a < na - 1:
            other[last] = a + 1
    return na, own, other


def _prolongator_matrix(P, nxn, nyn, B):
    """CSR matrix of the exported prolongator, and the mask of absent slots."""
    nn = nxn * nyn
    ncx, ownx, othx = _runs(nxn)
    ncy, owny, othy = _runs(nyn)
    P = P.reshape(4, B, 3, nn)
    jj, ii = np.divmod(np.arange(nn), nxn)
    rows, cols, vals, absent = [], [], [], []
    for s in range(4):
        Jx = ownx[ii] if s % 2 == 0 else othx[ii]
        Jy = owny[jj] if s // 2 == 0 else othy[jj]
        ok = (Jx >= 0) & (Jy >= 0)
        absent.append(P[s][:, :, ~ok].ravel())
        n = np.nonzero(ok)[0]
        J = Jy[n] * ncx + Jx[n]
        for r in range(B):
            for c in range(3):
                rows.append(B * n + r); cols.append(3 * J + c); vals.append(P[s, r, c, n])
    M = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(B * nn, 3 * ncx * ncy)).tocsr()
    M.sum_duplicates()
    return M, np.concatenate(absent)


@pytest.mark.parametrize("nx,ny,seed,prec", [(64, 48, 5, 0), (100, 37, 4, 0), (100, 37, 4, 1), (64, 48, 5, 2),
                                              (200, 40, 3, 1)])
def test_galerkin_coarse_operators(vp, nx, ny, seed, prec):
    """Every coarse operator equals P^T A P of the level above (exported through the
    C ABI and multiplied on the host), empty coarse dofs aside (unit diagonal), and
    prolongator entries of absent slots are zero.  In the FP32 and FP32 +
    BF16-coarse modes every product takes the FP32 copies of the level's A and P,
    with A P accumulated in FP32: FP32 rounding of inputs and of about 18-term
    (B = 2) or 27-term sums, times the cancellation of P^T A P, bounded here by 1e-5
    relative; the FP64 mode's products agree to 1e-12.  At 200 x 40 cells the finest
    row holds 67 aggregates, more than the 64 one workgroup of the FP32 first pass
    takes."""
    w, prob, ctx = _case(vp, nx, ny, seed)
    v = O.newton_solve(prob, maxit=2).v
    ctx.vp_newton_assemble(_dev(v.reshape(-1, 2)), _dev(prob.pi_consistent(v)), vp.VP_SVN)
    n, a, k = vp.default_opts()
    a.precision = prec
    ctx.vp_amg_setup(a)
    levels = ctx.vp_amg_info()
    print(f"[galerkin] levels {levels}", flush=True)
    assert len(levels) >= 3
    mats = []
    for l, (nxn, nyn, B) in enumerate(levels):
        At = torch.zeros(5 * B * B * nxn * nyn, dtype=torch.float64, device="cuda")
        Pt = torch.zeros(12 * B * nxn * nyn, dtype=torch.float64, device="cuda") if l + 1 < len(levels) else None
        ctx.vp_amg_export(l, At, Pt)
        mats.append((_host(At), None if Pt is None else _host(Pt)))
    for l in range(len(levels) - 1):
        nxn, nyn, B = levels[l]
        A = _stencil_matrix(mats[l][0], nxn, nyn, B)
        P, absent = _prolongator_matrix(mats[l][1], nxn, nyn, B)
        assert np.all(absent == 0.0)
        G = (P.T @ A @ P).toarray()
        d = np.diag(G).copy()
        d[d == 0.0] = 1.0
        np.fill_diagonal(G, d)
        cx, cy, cB = levels[l + 1]
        Ac = _stencil_matrix(mats[l + 1][0], cx, cy, cB).toarray()
        err = np.linalg.norm(Ac - G) / np.linalg.norm(G)
        print(f"[galerkin] prec {prec} level {l}->{l + 1}: rel err {err:.2e}", flush=True)
        assert err < (1e-5 if prec in (1, 2) else 1e-12)


def test_fp32_finest_prolongator_close_to_fp64(vp):
    """The FP32 modes smooth every prolongator from the FP32 operator and keep it in
    FP32 only (exported widened): the finest matches the FP64 mode's to FP32
    rounding (fresh contexts, so the spectral estimates start alike), and the next
    one, made from the first coarse operator, to the latter's difference."""
    nx, ny, seed = 100, 37, 4
    outs = {}
    for prec in (0, 1, 2):
        w, prob, ctx = _case(vp, nx, ny, seed)
        v = O.newton_solve(prob, maxit=2).v
        ctx.vp_newton_assemble(_dev(v.reshape(-1, 2)), _dev(prob.pi_consistent(v)), vp.VP_SVN)
        n, a, k = vp.default_opts()
        a.precision = prec
        ctx.vp_amg_setup(a)
        levels = ctx.vp_amg_info()
        Ps = []
        for l in range(2):
            nxn, nyn, B = levels[l]
            Pt = torch.zeros(12 * B * nxn * nyn, dtype=torch.float64, device="cuda")
            ctx.vp_amg_export(l, None, Pt)
            Ps.append(_host(Pt))
        outs[prec] = Ps
    for prec in (1, 2):
        d0 = _relerr(outs[prec][0], outs[0][0])
        d1 = _relerr(outs[prec][1], outs[0][1])
        f32 = all(np.array_equal(P, P.astype(np.float32).astype(np.float64)) for P in outs[prec])
        print(f"[prolongator] prec {prec}: finest rel diff {d0:.2e} (FP32 values: {f32}), next {d1:.2e}", flush=True)
        assert f32 and 0 < d0 < 1e-6
        assert d1 < 1e-5


_VC_CASES = {}


def _vcycle(vp, nx, ny, seed, prec, degree, rseed, variant=0, walk4_rows=0):
    """One V-cycle of a fresh context (so the spectral estimates are identical) on a
    random residual, with the given kernel variant flags and walk strip height."""
    key = (nx, ny, seed)
    if key not in _VC_CASES:
        w = inputs.synthetic(nx, seed, ny=ny, Ly=512e3 * ny / nx)
        w.v_prev = 0.05 * np.random.default_rng(seed).standard_normal(w.v_prev.shape)
        prob = O.problem_from_workload(w)
        v = _rand_v(prob, 3, 0.05)
        _VC_CASES[key] = (w, prob, v, prob.pi_consistent(v))
    w, prob, v, pi = _VC_CASES[key]
    print(f"[case] nx={nx} ny={ny} seed={seed} prec={prec} degree={degree} variant={variant} rows={walk4_rows}",
          flush=True)
    ctx = vp.context_for(w)
    ctx.vp_newton_assemble(_dev(v.reshape(-1, 2)), _dev(pi), vp.VP_SVN)
    rng = np.random.default_rng(rseed)
    r = rng.standard_normal(2 * prob.mesh.nnode)
    r[~prob.mesh.free_dof] = 0.0
    n, a, k = vp.default_opts()
    a.precision, a.cheb_degree, a.variant, a.walk4_rows = prec, degree, variant, walk4_rows
    ctx.vp_amg_setup(a)
    z = torch.zeros(prob.mesh.nnode, 2, dtype=torch.float64, device="cuda")
    ctx.vp_amg_apply(_dev(r.reshape(-1, 2)), z)
    return _host(z).ravel(), ctx


@pytest.mark.parametrize("prec", [0, 1, 2, 5, 6])
def test_vcycle_tail_kernel_matches_per_sweep_launches(vp, prec):
    """The single-workgroup kernel for the smallest levels runs the same per-node
    arithmetic as the one-launch-per-sweep path: the V-cycle outputs are bitwise
    equal (VP_AMG_VAR_NO_TAIL switches the single-workgroup kernel off at setup)."""
    ref, _ = _vcycle(vp, 200, 150, 8, prec, 4, 4, variant=vp.VP_AMG_VAR_NO_TAIL)
    out, ctx = _vcycle(vp, 200, 150, 8, prec, 4, 4)
    print(f"[tail] prec={prec} levels {ctx.vp_amg_info()} max |diff| {np.abs(ref - out).max():.2e}", flush=True)
    assert np.array_equal(ref, out)


@pytest.mark.parametrize("degree", [2, 3, 4, 5])
@pytest.mark.parametrize("prec", [0, 1, 2, 4, 5, 6])
def test_paired_sweeps_match_single_sweeps(vp, prec, degree):
    """The finest-level smoother with its sweeps fused (two Chebyshev steps per
    pass, or all four of a degree-4 smoothing in one column walk) gives bitwise the
    V-cycle of one launch per sweep (VP_AMG_VAR_NO_PAIRS), for even and odd step
    counts, in every storage mode with fused sweeps (BF16 coarse levels included)."""
    ref, _ = _vcycle(vp, 200, 150, 8, prec, degree, 5, variant=vp.VP_AMG_VAR_NO_PAIRS)
    out, _ = _vcycle(vp, 200, 150, 8, prec, degree, 5)
    print(f"[pairs] prec={prec} degree={degree} max |diff| {np.abs(ref - out).max():.2e} "
          f"|z| {np.abs(out).max():.2e}", flush=True)
    assert np.array_equal(ref, out)


@pytest.mark.parametrize("rows", [1, 5, 13, 38, 79, 151])
@pytest.mark.parametrize("prec", [0, 1])
def test_walk4_strip_heights(vp, prec, rows):
    """The four-sweep column walk gives bitwise the single sweeps' V-cycle for any
    strip height: short strips, the 38 (FP32) and 79 (FP64) rows the launcher picks
    at 2049^2, and one strip over the whole mesh (the halo rows each strip
    recomputes are the same).  Each workgroup walks its lower strip upward and its
    upper strip downward; odd strip counts leave an upper strip past the mesh."""
    ref, _ = _vcycle(vp, 200, 150, 8, prec, 4, 9, variant=vp.VP_AMG_VAR_NO_PAIRS)
    out, _ = _vcycle(vp, 200, 150, 8, prec, 4, 9, walk4_rows=rows)
    print(f"[walk4 rows] prec={prec} rows={rows} max |diff| {np.abs(ref - out).max():.2e}", flush=True)
    assert np.array_equal(ref, out)


@pytest.mark.parametrize("prec", [1, 2])
def test_walk4_production_geometry_2048(vp, prec):
    """At the benchmark's 2048^2 cells the launcher runs the walk in its production
    geometry (tall strips sized to the resident workgroups); the V-cycle is bitwise
    the one of single sweeps.  (v random, pi = tau/Delta of it, both set on the GPU.)"""
    n = 2048
    outs = []
    for variant in (vp.VP_AMG_VAR_NO_PAIRS, 0):
        w = inputs.synthetic(n, 10)
        print(f"[walk4 2048] prec={prec} variant={variant}", flush=True)
        ctx = vp.context_for(w)
        g = torch.Generator(device="cuda").manual_seed(3)
        v = 0.05 * torch.randn(ctx.node_shape, dtype=torch.float64, device="cuda", generator=g)
        vv = v.view(n + 1, n + 1, 2)
        vv[0].zero_(); vv[-1].zero_(); vv[:, 0].zero_(); vv[:, -1].zero_()
        pi = torch.zeros(ctx.pi_shape, dtype=torch.float64, device="cuda")
        ctx.vp_pi_init(v, pi)
        ctx.vp_newton_assemble(v, pi, vp.VP_SVN)
        _, a, _ = vp.default_opts()
        a.precision, a.variant = prec, variant
        ctx.vp_amg_setup(a)
        r = torch.randn(ctx.node_shape, dtype=torch.float64, device="cuda", generator=g)
        z = torch.zeros_like(r)
        ctx.vp_amg_apply(r, z)
        outs.append(_host(z).ravel())
        ctx.close()
        del ctx
        torch.cuda.empty_cache()
    print(f"[walk4 2048] prec={prec} max |diff| {np.abs(outs[0] - outs[1]).max():.2e}", flush=True)
    assert np.isfinite(outs[1]).all() and np.abs(outs[1]).max() > 0
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("degree", [2, 4])
@pytest.mark.parametrize("prec", [1, 2, 4, 6])
def test_lds_tail_matches_tail(vp, prec, degree):
    """The one-workgroup tail with FP32 vectors in LDS and each node's stencil blocks
    in registers gives bitwise the V-cycle of the tail that reloads everything from
    global memory every sweep (VP_AMG_VAR_NO_TAIL_LDS)."""
    ref, _ = _vcycle(vp, 200, 150, 8, prec, degree, 7, variant=vp.VP_AMG_VAR_NO_TAIL_LDS)
    out, _ = _vcycle(vp, 200, 150, 8, prec, degree, 7)
    print(f"[lds tail] prec={prec} degree={degree} max |diff| {np.abs(ref - out).max():.2e}", flush=True)
    assert np.array_equal(ref, out)


@pytest.mark.parametrize("degree", [3, 4])
@pytest.mark.parametrize("prec", [1, 2, 4, 6])
def test_coarse_paired_sweeps_match_single_sweeps(vp, prec, degree):
    """On a mesh whose first coarse level has over 10^5 nodes (961^2 -> 321^2) the
    coarse levels smooth with paired sweeps too (column walks for FP32 3 x 3 blocks,
    tiles for BF16 storage); the V-cycle is bitwise the one of single sweeps on every
    level."""
    ref, _ = _vcycle(vp, 960, 960, 9, prec, degree, 6, variant=vp.VP_AMG_VAR_NO_PAIRS)
    out, ctx = _vcycle(vp, 960, 960, 9, prec, degree, 6)
    levels = ctx.vp_amg_info()
    assert levels[1][0] * levels[1][1] >= 100000
    print(f"[coarse pairs] prec={prec} degree={degree} max |diff| {np.abs(ref - out).max():.2e}", flush=True)
    assert np.array_equal(ref, out)


@pytest.mark.parametrize("prec", [1, 2])
def test_fp32_copy_from_assembly_matches_conversion(vp, prec):
    """After a setup in an FP32 mode the next assembly also writes the FP32 copy of the
    operator that the setup would otherwise convert.  The two copies are bitwise
    equal: two Newton solves of the same inputs in one context (the first one's first
    step converts, every later step uses the assembly's copy) give bitwise the same
    velocity, dual field and iteration counts (a solve restarts its spectral
    estimates, so it is a function of its inputs only)."""
    w = inputs.sharp_step(160)
    ctx = vp.context_for(w)
    outs = []
    for rep in range(2):
        v = torch.zeros(ctx.node_shape, dtype=torch.float64, device="cuda")
        pi = torch.zeros(ctx.pi_shape, dtype=torch.float64, device="cuda")
        n, a, k = vp.default_opts()
        a.precision = prec
        rc, info, _ = ctx.vp_newton_solve(v, pi, 200, n, a, k, history=False)
        print(f"[fp32 copy] prec={prec} solve {rep}: rc={rc} its={info.iterations} krylov={info.krylov_iters}",
              flush=True)
        assert rc == 0
        outs.append((_host(v).copy(), _host(pi).copy(), info.iterations, info.krylov_iters))
    assert outs[0][2:] == outs[1][2:]
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
