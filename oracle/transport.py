"""Oracle for the explicit transport step of A and H (test infrastructure).

Only tests/, the smoke check and the benchmark's CPU baseline may import this
module.  Plain numpy FP64, written independently of the HIP kernels.

Eq. model:A and eq. model:H (Sec. 2) advanced by one explicit Euler step (Sec. 3)
with cell-wise constant A and H (finite volumes, the Q0-disc space of Sec. 5) on
the structured mesh and the Q1 velocity v:

  Q_c^{n+1} = Q_c^n - dt/|c| * sum over the faces f of c of  F_f,
  F_f = (v . n_f) |f| Q_up,

where v . n_f is the mean of the normal velocity along the face (the mean of the
face's two nodal values, exact for Q1; Simpson's rule on the face's three nodes for
Q2) and Q_up is the value of the cell the flow
comes from (first-order upwind).  The velocity vanishes on the boundary (zero
Dirichlet condition), so boundary faces carry no flux and the inflow values of
Sec. 2 never enter.  Readings: faces whose mean normal velocity is exactly 0 take
no flux; after the step A is clipped to [0, 1] and H to [0, inf) (the paper does
not say how over- or undershoots are treated).
"""
from __future__ import annotations

import numpy as np


def face_velocities(v, nx, ny, order=1):
    """Mean normal velocity on the vertical faces ux [ny][nx+1] (face between
    cells i-1 and i of row j at x = i hx) and horizontal faces uy [ny+1][nx].
    Q1 velocity: the mean of the face's two end values.  Q2 velocity (nodes at the
    face's ends and midpoint): Simpson's rule, exact for the quadratic trace."""
    if order == 1:
        V = np.asarray(v, dtype=np.float64).reshape(ny + 1, nx + 1, 2)
        ux = 0.5 * (V[:-1, :, 0] + V[1:, :, 0])
        uy = 0.5 * (V[:, :-1, 1] + V[:, 1:, 1])
    else:
        V = np.asarray(v, dtype=np.float64).reshape(2 * ny + 1, 2 * nx + 1, 2)
        Vx = V[:, ::2, 0]                      # columns at cell faces x = i hx
        ux = (Vx[0:-1:2] + 4.0 * Vx[1::2] + Vx[2::2]) / 6.0
        Vy = V[::2, :, 1]                      # rows at cell faces y = j hy
        uy = (Vy[:, 0:-1:2] + 4.0 * Vy[:, 1::2] + Vy[:, 2::2]) / 6.0
    ux[:, 0] = 0.0
    ux[:, nx] = 0.0
    uy[0, :] = 0.0
    uy[ny, :] = 0.0
    return ux, uy


def upwind_fluxes(Q, ux, uy, hx, hy):
    """Face fluxes (v.n)|f| Q_up: Fx [ny][nx+1] in +x, Fy [ny+1][nx] in +y."""
    ny, nx = Q.shape
    Fx = np.zeros((ny, nx + 1))
    Fy = np.zeros((ny + 1, nx))
    for i in range(1, nx):          # interior vertical faces
        left, right = Q[:, i - 1], Q[:, i]
        u = ux[:, i]
        Fx[:, i] = u * hy * np.where(u > 0.0, left, right)
    for j in range(1, ny):          # interior horizontal faces
        below, above = Q[j - 1, :], Q[j, :]
        u = uy[j, :]
        Fy[j, :] = u * hx * np.where(u > 0.0, below, above)
    return Fx, Fy


def advect(v, A, H, nx, ny, Lx, Ly, dt, clip=True, order=1):
    """One explicit upwind step of A and H ([ny][nx] arrays) with velocity v (Q1 or
    Q2 nodal values)."""
    hx, hy = Lx / nx, Ly / ny
    ux, uy = face_velocities(v, nx, ny, order)
    out = []
    for Q in (np.asarray(A, dtype=np.float64).reshape(ny, nx), np.asarray(H, dtype=np.float64).reshape(ny, nx)):
        Fx, Fy = upwind_fluxes(Q, ux, uy, hx, hy)
        div = (Fx[:, 1:] - Fx[:, :-1]) + (Fy[1:, :] - Fy[:-1, :])
        out.append(Q - dt / (hx * hy) * div)
    A1, H1 = out
    if clip:
        A1 = np.clip(A1, 0.0, 1.0)
        H1 = np.maximum(H1, 0.0)
    return A1, H1
