"""Pins of the oracle's Q2 (biquadratic) velocity elements (Sec. 5: the method with
higher-order elements), against the mathematics: exact reproduction of
biquadratic fields by the basis, exactness of the 3x3 Gauss rule, the gradient
identities of the Theorem (Sec. 3), the svN/stdN equivalence (Sec. 4.2),
symmetry and definiteness (Sec. 5.4), brute-force minimisation of the energy and
the convergence rate on a manufactured solution."""
import math

import numpy as np
import pytest
import scipy.optimize as so
import scipy.sparse.linalg as spla

from oracle import vp_oracle as O
from paper_2204_10822_amd import inputs


def _prob(n=3, seed=0, **kw):
    w = inputs.synthetic(n, 300 + seed, wind_max=15.0, delta_min=kw.pop("delta_min", 2e-9), order=2)
    d = w.desc.replace(**kw)
    rng = np.random.default_rng(seed)
    vp = 0.05 * rng.standard_normal(w.v_prev.shape)
    return O.VPProblem(d, w.H, w.A, w.v_air, w.v_ocean, vp)


def _rand_v(p, seed, scale=0.1):
    rng = np.random.default_rng(seed)
    v = scale * rng.standard_normal(2 * p.mesh.nnode)
    v[~p.mesh.free_dof] = 0.0
    return v


def test_q2_basis_reproduces_biquadratics_and_gauss_rule():
    nx, ny, Lx, Ly = 3, 2, 300e3, 170e3
    m = O.Mesh(nx, ny, Lx, Ly, order=2)
    assert (m.nxn, m.nyn, m.nen, m.nq) == (7, 5, 9, 9)
    # node coordinates on the (2nx+1) x (2ny+1) grid, computed here independently
    X, Y = np.meshgrid(np.linspace(0, Lx, 2 * nx + 1), np.linspace(0, Ly, 2 * ny + 1), indexing="xy")
    X, Y = X.ravel(), Y.ravel()
    f = lambda x, y: (1 + 2 * x / Lx - 3 * (x / Lx) ** 2) * (2 - y / Ly + 5 * (y / Ly) ** 2)
    fx = lambda x, y: (2 / Lx - 6 * x / Lx ** 2) * (2 - y / Ly + 5 * (y / Ly) ** 2)
    fy = lambda x, y: (1 + 2 * x / Lx - 3 * (x / Lx) ** 2) * (-1 / Ly + 10 * y / Ly ** 2)
    nodal = np.stack([f(X, Y), fy(X, Y)], -1)          # two biquadratic fields
    vals = m.at_corners(nodal)
    for j in range(ny):
        for i in range(nx):
            for q in range(m.nq):
                w, N, dx, dy = m.qp[q]
                # the quadrature point's physical position, from the basis itself
                xq = N @ X[m.corners[:, j, i]]
                yq = N @ Y[m.corners[:, j, i]]
                assert N.sum() == pytest.approx(1.0, abs=1e-14)
                assert N @ vals[:, j, i, 0] == pytest.approx(f(xq, yq), rel=1e-12)
                assert dx @ vals[:, j, i, 0] == pytest.approx(fx(xq, yq), rel=1e-10, abs=1e-18)
                assert dy @ vals[:, j, i, 0] == pytest.approx(fy(xq, yq), rel=1e-10, abs=1e-18)
    # the 3x3 Gauss rule integrates x^5 y^4 exactly over a cell
    x0, y0 = Lx / nx, 0.0
    tot = 0.0
    for q in range(m.nq):
        w, N, _, _ = m.qp[q]
        xq = N @ X[m.corners[:, 0, 1]]
        yq = N @ Y[m.corners[:, 0, 1]]
        tot += w * (xq / Lx) ** 5 * (yq / Ly) ** 4
    hx, hy = m.hx, m.hy
    exact = ((2 * hx / Lx) ** 6 - (hx / Lx) ** 6) / 6 * Lx * ((hy / Ly) ** 5 - 0) / 5 * Ly
    assert tot == pytest.approx(exact, rel=1e-12)


def test_q2_residual_is_energy_gradient():
    p = _prob(3, delta_min=1e-7)
    v = _rand_v(p, 3)
    R = p.residual(v, dirichlet=False)
    rng = np.random.default_rng(4)
    for _ in range(4):
        d = rng.standard_normal(v.size)
        h = 1e-6
        fd = (p.energy(v + h * d)[0] - p.energy(v - h * d)[0]) / (2 * h)
        assert fd == pytest.approx(R @ d, rel=1e-7)


def test_q2_std_jacobian_is_residual_derivative():
    p = _prob(3, delta_min=1e-7)
    v = _rand_v(p, 5)
    J = p.jacobian_std(v)
    rng = np.random.default_rng(6)
    d = rng.standard_normal(v.size)
    d[~p.mesh.free_dof] = 0.0
    h = 1e-5
    fd = (p.residual(v + h * d) - p.residual(v - h * d)) / (2 * h)
    Jd = J @ d
    assert np.linalg.norm(fd - Jd) <= 1e-6 * np.linalg.norm(Jd)


def test_q2_svn_equals_std_at_consistent_pi_and_is_spd():
    p = _prob(3)
    v = _rand_v(p, 7)
    Ks = p.jacobian_svn(v, p.pi_consistent(v))
    Kd = p.jacobian_std(v)
    assert spla.norm(Ks - Kd) <= 1e-13 * spla.norm(Kd)
    rng = np.random.default_rng(9)
    pi = 2.0 * rng.standard_normal((9, 3, 3, 3))
    K = p.jacobian_svn(v, pi).toarray()
    assert np.abs(K - K.T).max() <= 1e-14 * np.abs(K).max()
    np.linalg.cholesky(K)


def test_q2_newton_matches_bruteforce_minimisation():
    p = _prob(2, delta_min=3e-7)
    free = p.mesh.free_dof
    res = O.newton_solve(p, variant="svn", tol=1e-12)
    assert res.converged

    def f(x):
        v = np.zeros(free.size)
        v[free] = x
        return p.energy(v)[0]

    def g(x):
        v = np.zeros(free.size)
        v[free] = x
        return p.residual(v)[free]

    x0 = np.zeros(free.sum())
    scale = f(x0 + 0.01) - f(x0)
    sol = so.minimize(f, x0, jac=g, method="BFGS", options=dict(gtol=1e-10 * abs(scale) / 0.01, maxiter=5000))
    np.testing.assert_allclose(sol.x, res.v[free], rtol=1e-6, atol=1e-9)


def _lag(t):
    """1-D quadratic Lagrange basis at nodes 0, 1/2, 1 and its derivative (written here
    independently of the oracle)."""
    return (np.array([2 * (t - 0.5) * (t - 1), 4 * t * (1 - t), 2 * t * (t - 0.5)]),
            np.array([4 * t - 3, 4 - 8 * t, 4 * t - 1]))


def _mms_load_q2(p, U, L):
    """A(v*, phi_i) by 6x6 Gauss per cell with the exact v* and grad v*."""
    m, prm = p.mesh, p.prm
    xg, wg = np.polynomial.legendre.leggauss(6)
    xg, wg = 0.5 * (xg + 1), 0.5 * wg
    nxn = 2 * m.nx + 1
    out = np.zeros(((2 * m.ny + 1) * nxn, 2))
    k = math.pi / L
    jj, ii = np.meshgrid(np.arange(m.ny), np.arange(m.nx), indexing="ij")
    for a_y in range(6):
        for a_x in range(6):
            xi, eta, w = xg[a_x], xg[a_y], wg[a_x] * wg[a_y] * m.hx * m.hy
            X = (ii + xi) * m.hx
            Y = (jj + eta) * m.hy
            v = np.stack([U * np.sin(k * X) * np.sin(2 * k * Y), U * np.sin(2 * k * X) * np.sin(k * Y)], -1)
            G = np.empty(X.shape + (2, 2))
            G[..., 0, 0] = U * k * np.cos(k * X) * np.sin(2 * k * Y)
            G[..., 0, 1] = U * 2 * k * np.sin(k * X) * np.cos(2 * k * Y)
            G[..., 1, 0] = U * 2 * k * np.cos(2 * k * X) * np.sin(k * Y)
            G[..., 1, 1] = U * k * np.sin(2 * k * X) * np.cos(k * Y)
            S = O.vp_stress(O.strain_rate(G), p.P, prm)
            f = p.rhoH[..., None] * v + prm.dt * prm.C_ocean * prm.rho_ocean * np.linalg.norm(v, axis=-1)[..., None] * v
            lx, dlx = _lag(xi)
            ly, dly = _lag(eta)
            for by in range(3):
                for bx in range(3):
                    N = lx[bx] * ly[by]
                    dN = np.array([dlx[bx] * ly[by] / m.hx, lx[bx] * dly[by] / m.hy])
                    node = (2 * jj + by) * nxn + 2 * ii + bx
                    contrib = w * (N * f + prm.dt * np.einsum("yxdj,j->yxd", S, dN))
                    np.add.at(out, node.ravel(), contrib.reshape(-1, 2))
    return out.ravel()


def test_q2_manufactured_solution_rate():
    """Smooth viscous flow with a manufactured load: nodal errors fall at least with
    h^2.5 (the Q2 rate; Q1 shows h^2 on the same problem)."""
    L, U = 512e3, 0.1
    errs = []
    for n in (4, 8, 16):
        w = inputs.synthetic(n, 21, order=2)
        z = np.zeros_like(w.v_air)
        d = w.desc.replace(delta_min=1e-6, f_coriolis=0.0)
        H = np.full_like(w.H, 1.0)
        p0 = O.VPProblem(d, H, np.ones_like(H), z, z, z)
        b = _mms_load_q2(p0, U, L)
        b[~p0.mesh.free_dof] = 0.0
        p = O.VPProblem(d, H, np.ones_like(H), z, z, z, extra_load=b)
        res = O.newton_solve(p, variant="svn", tol=1e-11)
        assert res.converged
        X, Y = inputs.node_coords(2 * n, 2 * n, L, L)
        k = math.pi / L
        vs = np.stack([U * np.sin(k * X) * np.sin(2 * k * Y), U * np.sin(2 * k * X) * np.sin(k * Y)], -1).ravel()
        errs.append(np.sqrt(np.mean((res.v - vs) ** 2)))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    print("q2 mms errors", errs, "rates", rates)
    assert all(r > 2.5 for r in rates), (errs, rates)
