"""Pins of the classical-AMG oracle (oracle/rs_amg.py) against closed forms,
textbook results and library routines, independent of the oracle itself."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import rs_amg as R


def lap1d(n):
    return sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1], format="csr")


def lap2d(m, stencil=5, eps=1.0):
    """Dirichlet Laplacian on an m x m interior grid (5-point, or 9-point with
    anisotropy eps between x and y)."""
    I = sp.identity(m)
    T = lap1d(m)
    if stencil == 5:
        return sp.csr_matrix(sp.kron(I, T) + eps * sp.kron(T, I))
    # bilinear-element Laplacian (9-point)
    M1 = sp.diags([np.ones(m - 1), 4 * np.ones(m), np.ones(m - 1)], [-1, 0, 1]) / 6.0
    return sp.csr_matrix(sp.kron(M1, T) + eps * sp.kron(T, M1))


def graph_laplacian(A):
    """Zero-row-sum version of A: off-diagonals kept, diagonal = -(sum of off-diagonals)."""
    A = sp.csr_matrix(A, copy=True)
    A.setdiag(0.0)
    A.eliminate_zeros()
    return sp.csr_matrix(A - sp.diags(np.asarray(A.sum(axis=1)).ravel()))


def test_strength_hand_example():
    """Row 0: -a = (4, 1, 2) for columns (1, 2, 3): threshold 0.5 * 4 = 2 -> {1, 3};
    positive couplings are never strong; a diagonally dominant row (|row sum| >
    0.9 a_ii) has none."""
    A = sp.csr_matrix(np.array([
        [10.0, -4.0, -1.0, -2.0, 0.5],
        [-4.0, 5.0, 0.0, 0.0, 0.0],
        [-1.0, 0.0, 2.0, -0.5, 0.0],
        [-2.0, 0.0, -0.5, 3.0, 0.0],
        [0.5, 0.0, 0.0, 0.0, 1.0],
    ]))
    S = R.strength(A, theta=0.5).toarray()
    assert S[0].tolist() == [False, True, False, True, False]
    assert S[1].tolist() == [True, False, False, False, False]
    # row 2: row sum 0.5 <= 0.9 * 2, strong {0, 3}: -a = (1, 0.5) >= 0.5
    assert S[2].tolist() == [True, False, False, True, False]
    # row 4: only a positive coupling
    assert not S[4].any()
    # row 3: |row sum| = 0.5 <= 2.7; -a = (2, 0.5): only column 0 reaches 0.5 * 2
    assert S[3].tolist() == [True, False, False, False, False]
    # the diagonal-dominance rule: scale row 1's diagonal so |row sum| > 0.9 a_11
    A2 = A.tolil()
    A2[1, 1] = 50.0
    assert not R.strength(sp.csr_matrix(A2), theta=0.5)[1].toarray().any()
    # and switched off at max_row_sum = 1
    assert R.strength(sp.csr_matrix(A2), theta=0.5, max_row_sum=1.0)[1].toarray().any()


def test_rs_1d_laplacian_alternates_and_interpolates_linearly():
    """1-D Laplacian: every other point is C, F points take 1/2 from each C
    neighbour (1/2 from the single one at an end), and P^T A P is (1/2) tridiag(-1, 2, -1)."""
    n = 15
    A = lap1d(n)
    S = R.strength(A, theta=0.25, max_row_sum=1.0)
    cf = R.rs_first_pass(S)
    # no two neighbours are both C, every F point has a C neighbour
    assert not np.any((cf[:-1] == R.C_PT) & (cf[1:] == R.C_PT))
    for i in np.nonzero(cf == R.F_PT)[0]:
        assert (i > 0 and cf[i - 1] == R.C_PT) or (i < n - 1 and cf[i + 1] == R.C_PT)
    # lowest index first among equal measures: 1, 3, 5, ... are C (0 and 2 depend on 1)
    assert cf.tolist() == [0, 1] * 7 + [0]
    P = R.interpolation(A, S, cf).toarray()
    for i in np.nonzero(cf == R.F_PT)[0]:
        nb = [j for j in (i - 1, i + 1) if 0 <= j < n and cf[j] == R.C_PT]
        assert np.allclose(P[i][P[i] != 0], 0.5) and len(nb) == (P[i] != 0).sum()
    Ac = R.galerkin(A, sp.csr_matrix(P)).toarray()
    nc = Ac.shape[0]
    assert np.allclose(Ac, 0.5 * lap1d(nc).toarray(), atol=1e-14)


def test_rs_2d_laplacian_splitting_properties():
    """5-point Laplacian with theta = 0.25: symmetric strength, so the C points are
    an independent set and every F point has a strong C neighbour; the first pass
    gives the checkerboard-like splitting with about half the points C."""
    m = 17
    A = lap2d(m)
    S = R.strength(A, theta=0.25, max_row_sum=1.0)
    assert (S != S.T).nnz == 0
    cf = R.rs_first_pass(S)
    Sc = sp.coo_matrix(S)
    assert not np.any((cf[Sc.row] == R.C_PT) & (cf[Sc.col] == R.C_PT))
    for i in np.nonzero(cf == R.F_PT)[0]:
        js = S.indices[S.indptr[i]:S.indptr[i + 1]]
        assert np.any(cf[js] == R.C_PT)
    frac = (cf == R.C_PT).mean()
    assert 0.4 < frac < 0.6


@pytest.mark.parametrize("eps", [1.0, 0.05])
def test_interpolation_reproduces_constants(eps):
    """On a zero-row-sum matrix (a graph Laplacian of the 9-point anisotropic
    stencil, strong F-F couplings at theta = 0.5) every F row with C neighbours
    interpolates constants exactly, and the coarse operator keeps zero row sums."""
    A = graph_laplacian(lap2d(12, stencil=9, eps=eps))
    S = R.strength(A, theta=0.5, max_row_sum=1.0)
    cf = R.rs_first_pass(S)
    P = R.interpolation(A, S, cf)
    nz = np.diff(P.indptr) > 0
    assert nz.sum() > 0.9 * A.shape[0]
    ones = P @ np.ones(P.shape[1])
    assert np.allclose(ones[nz], 1.0, atol=1e-13)
    # isotropic case: some F point really has a strong F neighbour (the distribution term runs)
    has_ff = eps != 1.0
    for i in np.nonzero(cf == R.F_PT)[0]:
        js = S.indices[S.indptr[i]:S.indptr[i + 1]]
        has_ff |= bool(np.any(cf[js] == R.F_PT))
    assert has_ff
    Ac = R.galerkin(A, P)
    full = np.asarray(np.diff(P.indptr) > 0)
    # coarse row sums vanish when every fine row interpolates constants
    if full.all():
        assert np.abs(Ac @ np.ones(Ac.shape[0])).max() < 1e-12 * abs(Ac.diagonal()).max()


def test_multicolour_sweep_is_gauss_seidel_in_colour_order():
    """One forward multicolour sweep equals sequential Gauss-Seidel with the rows
    ordered by colour: x = (D + L)^{-1} (b - U x0) in that order (scipy triangular solve)."""
    rng = np.random.default_rng(0)
    A = lap2d(9, stencil=9, eps=0.3) + sp.identity(81) * 0.1
    A = sp.csr_matrix(A)
    col = R.greedy_colouring(A)
    assert R.is_valid_colouring(A, col)
    b = rng.standard_normal(81)
    x0 = rng.standard_normal(81)
    perm = np.argsort(col, kind="stable")
    Ap = sp.csr_matrix(A[perm][:, perm])
    L = sp.tril(Ap, format="csr")
    U = sp.triu(Ap, k=1, format="csr")
    xp = spla.spsolve_triangular(L, b[perm] - U @ x0[perm], lower=True)
    # the forward half, written out: relax each colour at once
    d = A.diagonal()
    x = x0.copy()
    for c in range(col.max() + 1):
        rows = np.nonzero(col == c)[0]
        x[rows] += (b[rows] - A[rows] @ x) / d[rows]
    assert np.allclose(x[perm], xp, rtol=1e-12, atol=1e-12)
    # the symmetric sweep is the forward sweep followed by the backward one
    y = R.sgs(A, b, x0, col, 1)
    Lb = sp.triu(Ap, format="csr")
    Ub = sp.tril(Ap, k=-1, format="csr")
    yp = spla.spsolve_triangular(Lb, b[perm] - Ub @ xp, lower=False)
    assert np.allclose(y[perm], yp, rtol=1e-12, atol=1e-12)


def test_vcycle_poisson_convergence_and_symmetry():
    """Classical AMG on the 2-D Poisson problem: V(1,1) with symmetric GS reduces
    the error by at least 5x per cycle (textbook rates are ~0.1), the V-cycle is a
    symmetric operator, and with the coarse level as the only level it is the
    exact inverse."""
    m = 31
    A = lap2d(m)
    H = R.RSHierarchy(A, theta=0.25, max_row_sum=1.0, sweeps=1, max_coarse=20)
    assert len(H.P) >= 3
    rng = np.random.default_rng(1)
    b = np.zeros(m * m)
    x = rng.standard_normal(m * m)
    e0 = np.sqrt(x @ (A @ x))
    for _ in range(5):
        x = x + H.vcycle(b - A @ x)
    rate = (np.sqrt(x @ (A @ x)) / e0) ** (1 / 5)
    assert rate < 0.2
    u, v = rng.standard_normal(m * m), rng.standard_normal(m * m)
    assert abs(u @ H.vcycle(v) - v @ H.vcycle(u)) < 1e-10 * abs(u @ H.vcycle(u))
    H1 = R.RSHierarchy(lap2d(5), max_coarse=1000)
    assert len(H1.P) == 0
    bb = rng.standard_normal(25)
    assert np.allclose(lap2d(5) @ H1.vcycle(bb), bb)


def test_rs_pcg_on_vp_operator():
    """The classical-AMG preconditioner with the paper's settings solves an svN
    system of the sea-ice operator (Krylov vs direct solve)."""
    from oracle import vp_oracle as O
    from paper_2204_10822_amd import inputs
    w = inputs.synthetic(16, 3)
    prob = O.VPProblem(w.desc, w.H, w.A, w.v_air, w.v_ocean, w.v_prev)
    v = O.newton_solve(prob, maxit=2).v
    pi = prob.pi_consistent(v)
    K = prob.jacobian_svn(v, pi).tocsr()
    b = -prob.residual(v)
    H = R.RSHierarchy(K, theta=0.5, sweeps=3, max_coarse=40)
    assert len(H.P) >= 2
    its = []
    x, info = spla.cg(K, b, M=H.operator(), rtol=1e-10, maxiter=200, callback=lambda xk: its.append(1))
    assert info == 0
    xd = spla.spsolve(K.tocsc(), b)
    assert np.linalg.norm(x - xd) <= 1e-7 * np.linalg.norm(xd)
    assert len(its) < 60
