"""Pin of the oracle's stress-velocity Newton step against the unreduced system.

The oracle forms the svN step in reduced form: the operator of eq. linearSVNewton
(with eq. modification) for the velocity update, then the dual update of
eq. tautilde (with the same modification) at the quadrature points.  Here the
step is computed the other way, straight from the two-field formulation of
Sec. 4.2 on tiny meshes:

* the nonlinear map of eq. newAv=f and eq. res=0 (momentum with
  B(v, pi, phi) = (P pi, tau(phi)) - (P/2, tr eps(phi)), and the pointwise
  r(pi, v) = pi Delta(v) - tau(v)) is written out with its own element loop;
* its Jacobian in (v, pi) comes from complex-step differentiation of that map,
  not from any hand-derived formula;
* in the velocity block of r' (eq. R'), the term 2 (tau_l (x) pi_l) tau(v~)/Delta
  is replaced as eq. modification says, by
  [(tau_l : tau(v~)) pi_l + (pi_l : tau(v~)) tau_l] / (Delta s),
  s = max(1, sqrt(2 pi_l:pi_l)), with (X (x) Y) Z = (X:Z) Y as in eq. R';
* the whole square system (free velocity dofs + 3 stress components per point) is
  solved densely.

Its velocity part must equal spsolve(jacobian_svn, -R(v_l)) and its stress part
pi_step(v_l, v~, pi_l), at random (v_l, pi_l) that are far from consistent and
include points where 2 pi:pi > 1 (the scaling active) and < 1.
"""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import vp_oracle as O
from paper_2204_10822_amd import inputs

G0, G1 = 0.5 - 0.5 / math.sqrt(3.0), 0.5 + 0.5 / math.sqrt(3.0)


class TinyTwoField:
    """Two-field (v, pi) residual of Sec. 4.2 on an nx x ny Q1 mesh, complex-safe."""

    def __init__(self, w):
        d = w.desc
        self.d = d
        self.nx, self.ny = d.nx, d.ny
        self.nxn = d.nx + 1
        self.hx, self.hy = d.Lx / d.nx, d.Ly / d.ny
        self.H = np.asarray(w.H, float).reshape(d.ny, d.nx)
        self.A = np.asarray(w.A, float).reshape(d.ny, d.nx)
        self.va = np.asarray(w.v_air, float).reshape(-1, 2)
        self.vo = np.asarray(w.v_ocean, float).reshape(-1, 2)
        self.vn = np.asarray(w.v_prev, float).reshape(-1, 2)
        nn = (d.nx + 1) * (d.ny + 1)
        jj, ii = np.divmod(np.arange(nn), d.nx + 1)
        self.free = ~((ii == 0) | (jj == 0) | (ii == d.nx) | (jj == d.ny))
        self.nn = nn

    def cell_nodes(self, ci, cj):
        sw = cj * self.nxn + ci
        return [sw, sw + 1, sw + self.nxn, sw + self.nxn + 1]

    def shapes(self, xi, eta):
        N = np.array([(1 - xi) * (1 - eta), xi * (1 - eta), (1 - xi) * eta, xi * eta])
        dx = np.array([-(1 - eta), 1 - eta, -eta, eta]) / self.hx
        dy = np.array([-(1 - xi), -xi, 1 - xi, xi]) / self.hy
        return N, dx, dy

    def tau(self, G):
        """tau = eps'/e + tr(eps)/2 I from the gradient G[c][d] = d v_c / d x_d."""
        e = self.d.e_ratio
        E = 0.5 * (G + G.T)
        tr = E[0, 0] + E[1, 1]
        return (E - 0.5 * tr * np.eye(2)) / e + 0.5 * tr * np.eye(2)

    def residual(self, v, pi):
        """v: [nn, 2]; pi: [4, 3, ny, nx] (xx, yy, xy).  Returns (momentum [nn, 2], r [4, 3, ny, nx])."""
        d = self.d
        dt = d.dt
        dtype = np.result_type(v, pi)
        mom = np.zeros((self.nn, 2), dtype=dtype)
        r = np.zeros((4, 3, self.ny, self.nx), dtype=dtype)
        wq = 0.25 * self.hx * self.hy
        for cj in range(self.ny):
            for ci in range(self.nx):
                nodes = self.cell_nodes(ci, cj)
                P = d.P_star * self.H[cj, ci] * math.exp(-d.C_strength * (1.0 - self.A[cj, ci]))
                rh = d.rho_ice * self.H[cj, ci]
                for q, (xi, eta) in enumerate(((G0, G0), (G1, G0), (G0, G1), (G1, G1))):
                    N, dx, dy = self.shapes(xi, eta)
                    vq = sum(N[a] * v[nodes[a]] for a in range(4))
                    G = np.array([[sum(dx[a] * v[nodes[a], c] for a in range(4)),
                                   sum(dy[a] * v[nodes[a], c] for a in range(4))] for c in range(2)])
                    T = self.tau(G)
                    delta = np.sqrt(d.delta_min ** 2 + 2.0 * np.sum(T * T))
                    p = pi[q, :, cj, ci]
                    PI = np.array([[p[0], p[2]], [p[2], p[1]]])
                    R = PI * delta - T
                    r[q, 0, cj, ci], r[q, 1, cj, ci], r[q, 2, cj, ci] = R[0, 0], R[1, 1], R[0, 1]
                    vnq = sum(N[a] * self.vn[nodes[a]] for a in range(4))
                    voq = sum(N[a] * self.vo[nodes[a]] for a in range(4))
                    vaq = sum(N[a] * self.va[nodes[a]] for a in range(4))
                    w = voq - vq
                    t_oc = d.C_ocean * d.rho_ocean * np.sqrt(w[0] ** 2 + w[1] ** 2) * w
                    t_at = d.C_air * d.rho_air * math.hypot(*vaq) * vaq
                    u = vnq - voq
                    cor = rh * d.f_coriolis * np.array([-u[1], u[0]])       # e_r x (v^n - v_o)
                    force = rh * vq - dt * t_oc - (rh * vnq - dt * cor + dt * t_at)
                    for a in range(4):
                        for c in range(2):
                            Gphi = np.zeros((2, 2))
                            Gphi[c] = (dx[a], dy[a])
                            Tphi = self.tau(Gphi)
                            tr_eps = Gphi[0, 0] + Gphi[1, 1]
                            B = P * np.sum(PI * Tphi) - 0.5 * P * tr_eps
                            mom[nodes[a], c] += wq * (force[c] * N[a] + dt * B)
        return mom, r

    def delta_tau(self, v):
        """Delta and tau at every point: [4, ny, nx], [4, ny, nx, 2, 2]."""
        D = np.zeros((4, self.ny, self.nx))
        T = np.zeros((4, self.ny, self.nx, 2, 2))
        for cj in range(self.ny):
            for ci in range(self.nx):
                nodes = self.cell_nodes(ci, cj)
                for q, (xi, eta) in enumerate(((G0, G0), (G1, G0), (G0, G1), (G1, G1))):
                    _, dx, dy = self.shapes(xi, eta)
                    G = np.array([[sum(dx[a] * v[nodes[a], c] for a in range(4)),
                                   sum(dy[a] * v[nodes[a], c] for a in range(4))] for c in range(2)])
                    T[q, cj, ci] = self.tau(G)
                    D[q, cj, ci] = math.sqrt(self.d.delta_min ** 2 + 2.0 * np.sum(T[q, cj, ci] ** 2))
        return D, T


def _comp(X):
    """symmetric 2x2 -> (xx, yy, xy)"""
    return np.array([X[0, 0], X[1, 1], X[0, 1]])


def _frob(a, b):
    """X:Y for symmetric tensors given as (xx, yy, xy) components."""
    return a[0] * b[0] + a[1] * b[1] + 2.0 * a[2] * b[2]


def block_step(sys_, v, pi):
    """The svN step from the unreduced two-field system (modified as in eq. modification)."""
    free_nodes = np.flatnonzero(sys_.free)
    nv = 2 * free_nodes.size
    npi = pi.size
    h = 1e-30

    def res_vec(vv, pp):
        m, r = sys_.residual(vv, pp)
        return np.concatenate([m[free_nodes].ravel(), r.ravel()])

    g0 = res_vec(v.astype(complex), pi.astype(complex)).real
    J = np.zeros((nv + npi, nv + npi))
    for k in range(nv):
        vv = v.astype(complex)
        vv[free_nodes[k // 2], k % 2] += 1j * h
        J[:, k] = res_vec(vv, pi.astype(complex)).imag / h
    for k in range(npi):
        pp = pi.astype(complex).ravel()
        pp[k] += 1j * h
        J[:, nv + k] = res_vec(v.astype(complex), pp.reshape(pi.shape)).imag / h
    # tau(v~) per point as a linear map of the free dofs: minus the r-rows' velocity
    # block at pi = 0 (then r = -tau(v))
    Tmap = np.zeros((npi, nv))
    for k in range(nv):
        vv = v.astype(complex)
        vv[free_nodes[k // 2], k % 2] += 1j * h
        Tmap[:, k] = -res_vec(vv, np.zeros_like(pi, dtype=complex))[nv:].imag / h
    D, T = sys_.delta_tau(v)
    # replace the velocity block of r' by its modified form, point by point
    Jr = J[nv:, :nv].copy()
    for q in range(4):
        for cj in range(sys_.ny):
            for ci in range(sys_.nx):
                rows = [np.ravel_multi_index((q, c, cj, ci), pi.shape) for c in range(3)]
                tl = _comp(T[q, cj, ci])
                pl = pi[q, :, cj, ci]
                dl = D[q, cj, ci]
                s = max(1.0, math.sqrt(2.0 * _frob(pl, pl)))
                Tt = Tmap[rows]                                    # [3, nv]: tau(v~) comps
                t_tt = _frob(tl, Tt)                               # tau_l : tau(v~)
                p_tt = _frob(pl, Tt)                               # pi_l : tau(v~)
                unmod = 2.0 * np.outer(pl, t_tt) / dl - Tt         # eq. R' as derived
                # the complex-step block must be exactly the unmodified eq. R'
                np.testing.assert_allclose(Jr[rows], unmod, rtol=1e-10, atol=1e-12 * np.abs(unmod).max())
                Jr[rows] = (np.outer(pl, t_tt) + np.outer(tl, p_tt)) / (dl * s) - Tt
    J[nv:, :nv] = Jr
    x = np.linalg.solve(J, -g0)
    dv = np.zeros_like(v)
    dv[free_nodes] = x[:nv].reshape(-1, 2)
    return dv, x[nv:].reshape(pi.shape)


@pytest.mark.parametrize("nx,ny,seed", [(2, 2, 0), (3, 2, 1), (3, 3, 2), (4, 4, 3)])
def test_svn_step_equals_unreduced_two_field_system(nx, ny, seed):
    rng = np.random.default_rng(100 + seed)
    w = inputs.synthetic(nx, 7 + seed, (0.1, 2.0), (0.7, 1.0), 15.0, 2e-9, ny=ny)
    # non-zero previous velocity and ocean so that every load term is active
    w.v_prev = 0.05 * rng.standard_normal(w.v_prev.shape)
    prob = O.problem_from_workload(w)
    sys_ = TinyTwoField(w)
    nn = prob.mesh.nnode
    v = 0.2 * rng.standard_normal((nn, 2))
    v[prob.mesh.boundary] = 0.0
    # pi far from tau/Delta; magnitudes spread so that 2 pi:pi straddles 1
    pi = rng.standard_normal((4, 3, ny, nx)) * rng.uniform(0.05, 1.2, size=(4, 1, ny, nx))
    s = np.sqrt(2.0 * (pi[:, 0] ** 2 + pi[:, 1] ** 2 + 2.0 * pi[:, 2] ** 2))
    assert (s > 1.0).any() and (s < 1.0).any()
    dv_blk, dpi_blk = block_step(sys_, v, pi)
    K = prob.jacobian_svn(v.ravel(), pi)
    R = prob.residual(v.ravel())
    dv = spla.spsolve(K.tocsc(), -R)
    assert np.linalg.norm(dv - dv_blk.ravel()) <= 1e-10 * np.linalg.norm(dv)
    dpi = prob.pi_step(v.ravel(), dv, pi)
    assert np.linalg.norm(dpi - dpi_blk) <= 1e-10 * np.linalg.norm(dpi)


def test_two_field_momentum_at_consistent_pi_is_the_oracle_residual():
    # with pi = tau(v)/Delta(v) the momentum part of the two-field map is R(v)
    # (eq. sigma-pi equals eq. sigma there; Sec. 4.2)
    rng = np.random.default_rng(9)
    w = inputs.synthetic(4, 11, (0.1, 2.0), (0.7, 1.0), 15.0, 2e-9, ny=3)
    w.v_prev = 0.05 * rng.standard_normal(w.v_prev.shape)
    prob = O.problem_from_workload(w)
    sys_ = TinyTwoField(w)
    v = 0.2 * rng.standard_normal((prob.mesh.nnode, 2))
    v[prob.mesh.boundary] = 0.0
    pi = prob.pi_consistent(v.ravel())
    mom, r = sys_.residual(v, pi)
    mom[~sys_.free] = 0.0
    R = prob.residual(v.ravel())
    assert np.linalg.norm(mom.ravel() - R) <= 1e-12 * np.linalg.norm(R)
    D, _ = sys_.delta_tau(v)
    assert np.abs(r).max() <= 1e-13 * D.max()
