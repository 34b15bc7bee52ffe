"""CPU oracle for the implicit viscous-plastic momentum step (test infrastructure).

This module is test infrastructure.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import it; the product path never does.
It shares no code with the HIP library: it is a plain, slow FP64 numpy/scipy
implementation written from the paper's definitions, using 2x2 tensors (not the
Mandel vectors the kernels use) and scipy sparse matrices.

What it computes (paper sections / equations):
  * ice strength P = P* H exp(-C(1-A))                      eq. ice-strength
  * VP stress sigma = 2 eta eps' + zeta tr(eps) I - P/2 I     Sec. 2 (rheology)
    with zeta = P/(2 Delta), eta = zeta / e^2, Delta from   eq. Delta
  * drag forces tau_atm, tau_ocean                           eq. force
  * the energy Phi                                           eq. energy
  * the residual A(v, phi) - F(phi)                          eq. A, eq. F
  * the standard Newton Jacobian                             eq. standardNewton1/2
  * the stress-velocity Newton operator with the symmetrising
    and unit-sphere modification                             eq. linearSVNewton,
                                                             eq. modification
  * the dual update                                          eq. tautilde
  * the Newton iteration with energy backtracking            Sec. 4, Sec. 5.1

Discretisation choices where the paper is silent (each is a stated reading):
  Q1 velocity (or Q2 with desc.order = 2, Sec. 5) on a uniform structured quad
  mesh with zero Dirichlet data on the whole boundary; Q0 (cellwise constant)
  A, H and so P and rho*H; Gauss quadrature with 2x2 points for Q1 and 3x3 for Q2
  for every term (so the residual is the exact gradient of the discrete energy);
  wind and ocean velocities as nodal fields of the velocity space interpolated to
  quadrature points; the auxiliary stress pi stored per quadrature point.

Array conventions: node vectors are [nyn*nxn, 2] (node n = j*nxn+i; nxn = nx+1 for
Q1, 2nx+1 for Q2), dof index 2n+c.  pi is [nq, 3 comps (xx, yy, xy), ny, nx]
(nq = 4 or 9); quadrature point q = qx + k*qy (k = 2 or 3 points per direction,
lower point first).
Parity pins: every function here is pinned by tests in tests/test_oracle_*.py.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

# Gauss rules on [0, 1]: 2 points (Q1) and 3 points (Q2).
_G = (0.5 - 0.5 / math.sqrt(3.0), 0.5 + 0.5 / math.sqrt(3.0))
_G3 = (0.5 - 0.5 * math.sqrt(0.6), 0.5, 0.5 + 0.5 * math.sqrt(0.6))
_W3 = (5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0)


def _lagrange1d(order, t):
    """Values and derivatives of the 1-D Lagrange basis of the given order on [0, 1]
    (nodes 0, 1 for order 1; 0, 1/2, 1 for order 2) at t."""
    if order == 1:
        return np.array([1.0 - t, t]), np.array([-1.0, 1.0])
    return (np.array([2.0 * (t - 0.5) * (t - 1.0), -4.0 * t * (t - 1.0), 2.0 * t * (t - 0.5)]),
            np.array([4.0 * t - 3.0, -8.0 * t + 4.0, 4.0 * t - 1.0]))


class Mesh:
    """Uniform structured mesh of [0,Lx]x[0,Ly] with nx x ny cells and Q1 (order 1)
    or Q2 (order 2, biquadratic: nodes at cell corners, edge midpoints and centres)
    velocity elements (Sec. 5: Q1 by default, Q2 as the higher-order option)."""

    def __init__(self, nx: int, ny: int, Lx: float, Ly: float, order: int = 1):
        assert order in (1, 2)
        self.order = order
        self.nx, self.ny, self.Lx, self.Ly = nx, ny, Lx, Ly
        self.hx, self.hy = Lx / nx, Ly / ny
        self.nxn, self.nyn = order * nx + 1, order * ny + 1
        self.nnode = self.nxn * self.nyn
        k = order + 1                      # nodes per direction in a cell
        self.nen = k * k                   # element nodes
        jj, ii = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
        base = (order * jj) * self.nxn + order * ii
        # element node a = ax + k*ay at global node (order*i + ax, order*j + ay) -> [nen, ny, nx]
        self.corners = np.stack([base + ay * self.nxn + ax for ay in range(k) for ax in range(k)])
        bj, bi = np.meshgrid(np.arange(self.nyn), np.arange(self.nxn), indexing="ij")
        self.boundary = ((bi == 0) | (bi == self.nxn - 1) | (bj == 0) | (bj == self.nyn - 1)).ravel()
        self.free_dof = np.repeat(~self.boundary, 2)
        # quadrature table: (weight, N[nen], dN/dx[nen], dN/dy[nen]) per point q = qx + nq1*qy
        pts, wts = (_G, (0.5, 0.5)) if order == 1 else (_G3, _W3)
        self.qp = []
        for qy in range(len(pts)):
            for qx in range(len(pts)):
                lx, dlx = _lagrange1d(order, pts[qx])
                ly, dly = _lagrange1d(order, pts[qy])
                N = np.array([lx[ax] * ly[ay] for ay in range(k) for ax in range(k)])
                dx = np.array([dlx[ax] * ly[ay] for ay in range(k) for ax in range(k)]) / self.hx
                dy = np.array([lx[ax] * dly[ay] for ay in range(k) for ax in range(k)]) / self.hy
                self.qp.append((wts[qx] * wts[qy] * self.hx * self.hy, N, dx, dy))
        self.nq = len(self.qp)

    def at_corners(self, nodal: np.ndarray) -> np.ndarray:
        """nodal [nnode, k] -> [nen, ny, nx, k] (values at each cell's element nodes)"""
        return nodal.reshape(self.nnode, -1)[self.corners]

    def interp(self, corner_vals: np.ndarray, q: int) -> np.ndarray:
        N = self.qp[q][1]
        return np.einsum("a,a...->...", N, corner_vals)

    def grad(self, corner_vals: np.ndarray, q: int) -> np.ndarray:
        """Velocity gradient G[..., c, d] = d v_c / d x_d at point q."""
        _, _, dx, dy = self.qp[q]
        gx = np.einsum("a,a...->...", dx, corner_vals)
        gy = np.einsum("a,a...->...", dy, corner_vals)
        return np.stack([gx, gy], axis=-1)


@dataclass
class Params:
    rho_ice: float
    rho_air: float
    rho_ocean: float
    C_air: float
    C_ocean: float
    P_star: float
    C_strength: float
    e_ratio: float
    f_coriolis: float
    dt: float
    delta_min: float

    @staticmethod
    def from_desc(d) -> "Params":
        return Params(d.rho_ice, d.rho_air, d.rho_ocean, d.C_air, d.C_ocean, d.P_star,
                      d.C_strength, d.e_ratio, d.f_coriolis, d.dt, d.delta_min)


# ----------------------------------------------------------------------------
# pointwise constitutive pieces (Sec. 2 and Sec. 4)
# ----------------------------------------------------------------------------
_I2 = np.eye(2)


def ice_strength(H, A, prm: Params):
    """P = P* H exp(-C (1 - A))   (eq. ice-strength)."""
    return prm.P_star * H * np.exp(-prm.C_strength * (1.0 - A))


def strain_rate(G):
    """eps = (grad v + grad v^T) / 2 for gradients G[..., c, d]."""
    return 0.5 * (G + np.swapaxes(G, -1, -2))


def trace(M):
    return M[..., 0, 0] + M[..., 1, 1]


def deviator(E):
    return E - 0.5 * trace(E)[..., None, None] * _I2


def frob(X, Y):
    return np.einsum("...ij,...ij->...", X, Y)


def delta_of_strain(E, prm: Params):
    """Delta = sqrt(2 e^-2 eps':eps' + tr(eps)^2 + Delta_min^2)   (eq. Delta)."""
    Ed = deviator(E)
    return np.sqrt(2.0 * frob(Ed, Ed) / prm.e_ratio ** 2 + trace(E) ** 2 + prm.delta_min ** 2)


def tau_of_strain(E, prm: Params):
    """tau = e^-1 eps' + tr(eps)/2 I   (Sec. 4, start)."""
    return deviator(E) / prm.e_ratio + 0.5 * trace(E)[..., None, None] * _I2


def delta_of_tau(T, prm: Params):
    """Delta = sqrt(Delta_min^2 + 2 tau:tau)   (Sec. 4, start)."""
    return np.sqrt(prm.delta_min ** 2 + 2.0 * frob(T, T))


def vp_stress(E, P, prm: Params):
    """sigma = 2 eta eps' + zeta tr(eps) I - P/2 I, zeta = P/(2 Delta), eta = zeta e^-2."""
    D = delta_of_strain(E, prm)
    zeta = P / (2.0 * D)
    eta = zeta / prm.e_ratio ** 2
    return (2.0 * eta)[..., None, None] * deviator(E) \
        + (zeta * trace(E) - 0.5 * P)[..., None, None] * _I2


def ocean_stress(v, vo, prm: Params):
    """tau_ocean = C_o rho_o |v_o - v| (v_o - v)   (eq. force)."""
    w = vo - v
    return prm.C_ocean * prm.rho_ocean * np.linalg.norm(w, axis=-1)[..., None] * w


def air_stress(va, prm: Params):
    """tau_atm = C_a rho_a |v_a| v_a   (eq. force)."""
    return prm.C_air * prm.rho_air * np.linalg.norm(va, axis=-1)[..., None] * va


def e_r_cross(u):
    """e_r x u for the vertical unit vector e_r: (-u_y, u_x)."""
    return np.stack([-u[..., 1], u[..., 0]], axis=-1)


# ----------------------------------------------------------------------------
# the discrete problem
# ----------------------------------------------------------------------------
class VPProblem:
    """One implicit Euler momentum step (Sec. 3) on a Q1 mesh."""

    def __init__(self, desc, H, A, v_air, v_ocean, v_prev, extra_load=None):
        self.desc = desc
        self.prm = Params.from_desc(desc)
        self.mesh = Mesh(desc.nx, desc.ny, desc.Lx, desc.Ly, getattr(desc, "order", 1))
        m = self.mesh
        self.H = np.asarray(H, float).reshape(m.ny, m.nx)
        self.A = np.asarray(A, float).reshape(m.ny, m.nx)
        self.P = ice_strength(self.H, self.A, self.prm)
        self.rhoH = self.prm.rho_ice * self.H
        self.va_c = m.at_corners(np.asarray(v_air, float).reshape(-1, 2))
        self.vo_c = m.at_corners(np.asarray(v_ocean, float).reshape(-1, 2))
        self.vn_c = m.at_corners(np.asarray(v_prev, float).reshape(-1, 2))
        self.extra_load = None if extra_load is None else np.asarray(extra_load, float).ravel()
        self._tables()

    # --- basis-function tensors per quadrature point -------------------------
    def _tables(self):
        """For phi = N_a e_d: grad phi, eps(phi), tau(phi) per point: [nen, 2, 2, 2]."""
        m, prm = self.mesh, self.prm
        self.grad_phi, self.eps_phi, self.tau_phi = [], [], []
        for q in range(m.nq):
            _, N, dx, dy = m.qp[q]
            Gp = np.zeros((m.nen, 2, 2, 2))
            for a in range(m.nen):
                for d in range(2):
                    Gp[a, d, d, 0] = dx[a]
                    Gp[a, d, d, 1] = dy[a]
            Ep = strain_rate(Gp)
            self.grad_phi.append(Gp)
            self.eps_phi.append(Ep)
            self.tau_phi.append(tau_of_strain(Ep, prm))

    def _scatter_vec(self, elem):
        """element vectors [nen, ny, nx, 2] -> node vector [nnode*2]."""
        m = self.mesh
        out = np.zeros((m.nnode, 2))
        for a in range(m.nen):
            np.add.at(out, m.corners[a].ravel(), elem[a].reshape(-1, 2))
        return out.ravel()

    def qp_state(self, v, q):
        m = self.mesh
        vc = m.at_corners(np.asarray(v, float).reshape(-1, 2))
        return m.interp(vc, q), m.grad(vc, q)

    # --- F(phi)  (eq. F) -------------------------------------------------------
    def load(self):
        m, prm = self.mesh, self.prm
        elem = np.zeros((m.nen, m.ny, m.nx, 2))
        for q in range(m.nq):
            w, N, _, _ = m.qp[q]
            vn = m.interp(self.vn_c, q)
            vo = m.interp(self.vo_c, q)
            va = m.interp(self.va_c, q)
            f = self.rhoH[..., None] * vn \
                - prm.dt * self.rhoH[..., None] * prm.f_coriolis * e_r_cross(vn - vo) \
                + prm.dt * air_stress(va, prm)
            elem += w * N[:, None, None, None] * f[None]
        F = self._scatter_vec(elem)
        if self.extra_load is not None:
            F = F + self.extra_load
        return F

    # --- A(v, phi) - F(phi)  (eq. A and eq. F) -------------------------------
    def residual(self, v, dirichlet=True):
        m, prm = self.mesh, self.prm
        elem = np.zeros((m.nen, m.ny, m.nx, 2))
        for q in range(m.nq):
            w, N, _, _ = m.qp[q]
            vq, G = self.qp_state(v, q)
            E = strain_rate(G)
            S = vp_stress(E, self.P, prm)                      # [ny, nx, 2, 2]
            vo = m.interp(self.vo_c, q)
            f = self.rhoH[..., None] * vq - prm.dt * ocean_stress(vq, vo, prm)
            # (sigma, grad phi) for phi = N_a e_d
            elem += w * prm.dt * np.einsum("yxij,adij->ayxd", S, self.grad_phi[q])
            elem += w * N[:, None, None, None] * f[None]
        R = self._scatter_vec(elem) - self.load()
        if dirichlet:
            R[~m.free_dof] = 0.0
        return R

    # --- Phi(v)  (eq. energy) --------------------------------------------------
    def energy_terms(self, v):
        """Per-cell energy integrated by the element's Gauss rule: [ny, nx]."""
        m, prm = self.mesh, self.prm
        out = np.zeros((m.ny, m.nx))
        for q in range(m.nq):
            w = m.qp[q][0]
            vq, G = self.qp_state(v, q)
            E = strain_rate(G)
            vn = m.interp(self.vn_c, q)
            vo = m.interp(self.vo_c, q)
            va = m.interp(self.va_c, q)
            wv = vo - vq
            dens = 0.5 * self.rhoH * (vq * vq).sum(-1) \
                - self.rhoH * (vn * vq).sum(-1) \
                + prm.dt * (0.5 * self.P * (delta_of_strain(E, prm) - trace(E))
                            + prm.C_ocean * prm.rho_ocean * np.linalg.norm(wv, axis=-1) ** 3 / 3.0) \
                + prm.dt * (self.rhoH * prm.f_coriolis * (e_r_cross(vn - vo) * vq).sum(-1)
                            - (air_stress(va, prm) * vq).sum(-1))
            out += w * dens
        if self.extra_load is not None:
            out = out.copy()
            out.flat[0] -= float(self.extra_load @ np.asarray(v, float).ravel())
        return out

    def energy(self, v):
        t = self.energy_terms(v)
        return math.fsum(t.ravel()), math.fsum(np.abs(t).ravel())

    # --- linearised operators ---------------------------------------------------
    def _assemble(self, elem):
        """element matrices [ny, nx, nen, 2, nen, 2] -> CSR with identity Dirichlet rows/cols."""
        m = self.mesh
        ne = 2 * m.nen
        dof = (2 * m.corners[:, :, :, None] + np.arange(2)).transpose(1, 2, 0, 3)  # [ny,nx,nen,2]
        dof = dof.reshape(m.ny, m.nx, ne)
        rows = np.broadcast_to(dof[:, :, :, None], (m.ny, m.nx, ne, ne)).ravel()
        cols = np.broadcast_to(dof[:, :, None, :], (m.ny, m.nx, ne, ne)).ravel()
        n = 2 * m.nnode
        K = sp.coo_matrix((elem.reshape(m.ny, m.nx, ne, ne).ravel(), (rows, cols)), shape=(n, n)).tocsr()
        f = m.free_dof.astype(float)
        Df = sp.diags(f)
        K = (Df @ K @ Df + sp.diags(1.0 - f)).tocsr()
        K.sum_duplicates()
        return K

    def _mass_drag_elem(self, v, q, elem):
        m, prm = self.mesh, self.prm
        w, N, _, _ = m.qp[q]
        vq, _ = self.qp_state(v, q)
        vo = m.interp(self.vo_c, q)
        wv = vo - vq
        nw = np.linalg.norm(wv, axis=-1)
        safe = np.where(nw > 0.0, nw, 1.0)
        # -dt tau_ocean'(v)(dv, phi) of eq. standardNewton2, plus the mass term
        rank1 = np.where((nw > 0.0)[..., None, None],
                         wv[..., :, None] * wv[..., None, :] / safe[..., None, None], 0.0)
        Mq = self.rhoH[..., None, None] * _I2 \
            + prm.dt * prm.C_ocean * prm.rho_ocean * (nw[..., None, None] * _I2 + rank1)
        NN = np.outer(N, N)
        elem += w * np.einsum("ab,yxdf->yxadbf", NN, Mq)

    def jacobian_std(self, v):
        """Standard Newton operator (eq. standardNewton1, standardNewton2)."""
        m, prm = self.mesh, self.prm
        elem = np.zeros((m.ny, m.nx, m.nen, 2, m.nen, 2))
        for q in range(m.nq):
            w = m.qp[q][0]
            _, G = self.qp_state(v, q)
            T = tau_of_strain(strain_rate(G), prm)
            D = delta_of_tau(T, prm)
            Tp = self.tau_phi[q]                               # [nen,2,2,2]
            tt = np.einsum("adij,bfij->adbf", Tp, Tp)          # tau(phi_b):tau(phi_a)
            Tl = np.einsum("yxij,adij->yxad", T, Tp)           # tau_l : tau(phi)
            c1 = prm.dt * self.P / D
            c2 = prm.dt * 2.0 * self.P / D ** 3
            elem += w * (c1[..., None, None, None, None] * tt[None, None]
                         - c2[..., None, None, None, None] * Tl[..., :, :, None, None] * Tl[..., None, None, :, :])
            self._mass_drag_elem(v, q, elem)
        return self._assemble(elem)

    def jacobian_svn(self, v, pi):
        """Stress-velocity Newton operator (eq. linearSVNewton) with tau_l (x) pi_l
        replaced by (tau_l (x) pi_l + pi_l (x) tau_l) / (2 max(1, sqrt(2 pi:pi)))
        (eq. modification), where (X (x) Y) Z = (X:Z) Y."""
        m, prm = self.mesh, self.prm
        elem = np.zeros((m.ny, m.nx, m.nen, 2, m.nen, 2))
        PI = pi_tensor(pi)
        for q in range(m.nq):
            w = m.qp[q][0]
            _, G = self.qp_state(v, q)
            T = tau_of_strain(strain_rate(G), prm)
            D = delta_of_tau(T, prm)
            Pq = PI[q]
            s = np.maximum(1.0, np.sqrt(2.0 * frob(Pq, Pq)))
            Tp = self.tau_phi[q]
            tt = np.einsum("adij,bfij->adbf", Tp, Tp)
            Tl = np.einsum("yxij,adij->yxad", T, Tp)           # tau_l : tau(phi_a)
            Pl = np.einsum("yxij,adij->yxad", Pq, Tp)          # pi_l  : tau(phi_a)
            c1 = prm.dt * self.P / D
            c2 = prm.dt * 2.0 * self.P / (D ** 2 * 2.0 * s)
            # test phi_a (row), trial dv = phi_b (column):
            # [(tau_l:tau(dv)) pi_l + (pi_l:tau(dv)) tau_l] : tau(phi)
            sym = Tl[..., None, None, :, :] * Pl[..., :, :, None, None] \
                + Pl[..., None, None, :, :] * Tl[..., :, :, None, None]
            elem += w * (c1[..., None, None, None, None] * tt[None, None]
                         - c2[..., None, None, None, None] * sym)
            self._mass_drag_elem(v, q, elem)
        return self._assemble(elem)

    # --- dual variable ---------------------------------------------------------
    def pi_consistent(self, v):
        """pi = tau(v)/Delta(v) at every quadrature point (eq. pi)."""
        m, prm = self.mesh, self.prm
        out = np.zeros((m.nq, 3, m.ny, m.nx))
        for q in range(m.nq):
            _, G = self.qp_state(v, q)
            T = tau_of_strain(strain_rate(G), prm)
            X = T / delta_of_tau(T, prm)[..., None, None]
            out[q] = pi_components(X)
        return out

    def pi_step(self, v, dv, pi):
        """Dual Newton step from eq. tautilde with the modification of eq. modification:
        pi~ = -pi_l + tau_l/D + tau(dv)/D - [(tau_l:tau(dv)) pi_l + (pi_l:tau(dv)) tau_l]/(D^2 s)."""
        m, prm = self.mesh, self.prm
        out = np.zeros((m.nq, 3, m.ny, m.nx))
        PI = pi_tensor(pi)
        for q in range(m.nq):
            _, G = self.qp_state(v, q)
            _, Gd = self.qp_state(dv, q)
            T = tau_of_strain(strain_rate(G), prm)
            Td = tau_of_strain(strain_rate(Gd), prm)
            D = delta_of_tau(T, prm)[..., None, None]
            Pq = PI[q]
            s = np.maximum(1.0, np.sqrt(2.0 * frob(Pq, Pq)))[..., None, None]
            mod = (frob(T, Td)[..., None, None] * Pq + frob(Pq, Td)[..., None, None] * T) / (2.0 * s)
            X = -Pq + T / D + Td / D - 2.0 * mod / D ** 2
            out[q] = pi_components(X)
        return out


def pi_tensor(pi):
    """[nq, 3, ny, nx] (xx, yy, xy) -> [nq, ny, nx, 2, 2] symmetric tensors."""
    pi = np.asarray(pi, float)
    T = np.empty(pi.shape[:1] + pi.shape[2:] + (2, 2))
    T[..., 0, 0] = pi[:, 0]
    T[..., 1, 1] = pi[:, 1]
    T[..., 0, 1] = pi[:, 2]
    T[..., 1, 0] = pi[:, 2]
    return T


def pi_components(X):
    """[.., 2, 2] -> [3, ..] with (xx, yy, symmetric xy)."""
    return np.stack([X[..., 0, 0], X[..., 1, 1], 0.5 * (X[..., 0, 1] + X[..., 1, 0])])


# ----------------------------------------------------------------------------
# Newton iteration (Sec. 4.2 and Sec. 5.1)
# ----------------------------------------------------------------------------
@dataclass
class NewtonResult:
    v: np.ndarray
    pi: np.ndarray
    converged: bool
    iterations: int
    history: list
    status: str


def line_search_accept(phi_new, phi_old, floor, rn_new, rn_old):
    """Backtracking acceptance on the energy (Sec. 5.1): accept a clear decrease,
    reject a clear increase; inside the round-off band |dPhi| <= floor the
    residual-norm decrease decides (the paper reports that residual-norm
    backtracking behaves alike)."""
    d = phi_new - phi_old
    if d < -floor:
        return True
    if d > floor:
        return False
    return rn_new < rn_old


def eisenstat_walker(rn, rn_prev, eta_prev, tol_abs, eta_max=0.1, gamma=0.9):
    """Inner relative tolerance: Eisenstat-Walker choice 2 with safeguard, capped at
    eta_max and floored at 0.5 * (target residual) / (current residual), Kelley's
    safeguard against oversolving the last linear system (the paper leaves the
    inner tolerance open)."""
    if rn_prev is None:
        eta = eta_max
    else:
        eta = gamma * (rn / rn_prev) ** 2
        sg = gamma * eta_prev ** 2
        if sg > 0.1:
            eta = max(eta, sg)
    eta = max(eta, 0.5 * tol_abs / rn)
    return min(eta, eta_max)


def newton_solve(prob: VPProblem, v0=None, pi0=None, variant="svn", tol=1e-8, maxit=200,
                 inner="direct", max_halvings=30, ls="energy", eta_max=0.1, amg=None,
                 verbose=False):
    m = prob.mesh
    n = 2 * m.nnode
    v = np.zeros(n) if v0 is None else np.asarray(v0, float).ravel().copy()
    v[~m.free_dof] = 0.0
    pi = prob.pi_consistent(v) if pi0 is None else np.asarray(pi0, float).copy()
    r0 = np.linalg.norm(prob.residual(np.zeros(n)))
    tol_abs = tol * r0
    hist = []
    R = prob.residual(v)
    rn = np.linalg.norm(R)
    phi, phi_abs = prob.energy(v)
    rn_prev, eta = None, eta_max
    for it in range(maxit + 1):
        hist.append(dict(it=it, rnorm=rn, rel=rn / r0 if r0 > 0 else 0.0, energy=phi))
        if verbose:
            print(f"[oracle] it {it:3d} |R|/|R0| {rn / max(r0, 1e-300):.3e} Phi {phi:.12e}")
        if rn <= tol_abs:
            return NewtonResult(v, pi, True, it, hist, "converged")
        if it == maxit:
            break
        K = prob.jacobian_std(v) if variant == "std" else prob.jacobian_svn(v, pi)
        if inner == "direct":
            dv = spla.spsolve(K.tocsc(), -R)
            kits = 0
        else:
            eta = eisenstat_walker(rn, rn_prev, eta, tol_abs, eta_max)
            from .sa_amg import SAAMG, pcg
            M = SAAMG(K, m.nxn, m.nyn, m.hx, m.hy, m.boundary) if amg is None else amg(K)
            dv, kits = pcg(K, -R, M, rtol=eta)
        hist[-1]["krylov_iters"] = kits
        alpha, accepted = 1.0, False
        for _ in range(max_halvings + 1):
            vt = v + alpha * dv
            Rt = prob.residual(vt)
            rnt = np.linalg.norm(Rt)
            if ls == "residual":
                ok = rnt < rn
            else:
                phit, phit_abs = prob.energy(vt)
                ok = line_search_accept(phit, phi, 1e-14 * max(phi_abs, phit_abs), rnt, rn)
            if ok:
                accepted = True
                break
            alpha *= 0.5
        hist[-1]["alpha"] = alpha
        if not accepted:
            return NewtonResult(v, pi, False, it, hist, "linesearch_fail")
        if variant == "svn":
            pi = pi + alpha * prob.pi_step(v, dv, pi)
        v = vt
        R, rn_prev, rn = Rt, rn, rnt
        phi, phi_abs = prob.energy(v)
        if variant == "std":
            pi = prob.pi_consistent(v)
    return NewtonResult(v, pi, False, maxit, hist, "not_converged")


def problem_from_workload(w, extra_load=None) -> VPProblem:
    return VPProblem(w.desc, w.H, w.A, w.v_air, w.v_ocean, w.v_prev, extra_load)
