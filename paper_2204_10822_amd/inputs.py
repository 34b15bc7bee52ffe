"""Seeded synthetic inputs for the implicit viscous-plastic momentum step.

This module produces problem descriptions and input fields only; it holds none of
the solver's arithmetic (no strain rates, viscosities, residuals or operators), so
both the HIP path and the CPU oracle may draw their inputs from it.

Fields follow the structure of the paper's test problems (Sec. 5.2 and 5.3): a
512 km square, a time step of half an hour, Table "tab:params" for the physics
constants, smooth thickness and concentration fields, a rotating ocean gyre and
Gaussian-shaped atmospheric vortices with an inflow angle of 72 degrees.  The
paper's own analytic Problem I fields (Sec. 5.2) are also provided.

Layouts (all numpy float64, C order):
  cell fields   H, A          [ny][nx]
  node fields   v_air, v_ocean, v_prev   [ny+1][nx+1][2]   (x component first);
                [2ny+1][2nx+1][2] for Q2 velocity elements (desc.order = 2)
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class ProblemDesc:
    """Mesh, physics constants and step settings (Table tab:params, Sec. 5.2/5.3).

    P_star: the table prints 27.5 N/m^2; the standard Hibler value 27.5 kN/m^2
    (27500 N/m^2) is used, as the workloads here state.  f_coriolis: the paper's
    runs use 0; the workloads here switch on a polar value that enters only the
    explicit right-hand side (Sec. 3 footnote), so the operator stays symmetric.
    """

    nx: int
    ny: int
    Lx: float = 512e3
    Ly: float = 512e3
    rho_ice: float = 900.0
    rho_air: float = 1.3
    rho_ocean: float = 1026.0
    C_air: float = 1.2e-3
    C_ocean: float = 5.5e-3
    P_star: float = 27500.0
    C_strength: float = 20.0
    e_ratio: float = 2.0
    f_coriolis: float = 1.46e-4
    dt: float = 1800.0
    delta_min: float = 2e-9
    order: int = 1          # velocity elements: 1 = Q1, 2 = Q2 (biquadratic), Sec. 5

    def replace(self, **kw) -> "ProblemDesc":
        return dataclasses.replace(self, **kw)


def node_coords(nx: int, ny: int, Lx: float, Ly: float):
    x = np.linspace(0.0, Lx, nx + 1)
    y = np.linspace(0.0, Ly, ny + 1)
    return np.meshgrid(x, y, indexing="xy")  # each [ny+1][nx+1]


def cell_centres(nx: int, ny: int, Lx: float, Ly: float):
    x = (np.arange(nx) + 0.5) * (Lx / nx)
    y = (np.arange(ny) + 0.5) * (Ly / ny)
    return np.meshgrid(x, y, indexing="xy")  # each [ny][nx]


def smooth_field(seed: int, nx: int, ny: int, Lx: float, Ly: float,
                 lo: float, hi: float, n_modes: int = 8) -> np.ndarray:
    """Sum of seeded cosine modes (integer wavenumbers 1..4 per direction),
    evaluated at cell centres and rescaled affinely onto [lo, hi]."""
    rng = np.random.default_rng(seed)
    X, Y = cell_centres(nx, ny, Lx, Ly)
    f = np.zeros((ny, nx))
    for _ in range(n_modes):
        kx, ky = rng.integers(1, 5, size=2)
        amp = rng.standard_normal() / math.hypot(kx, ky)
        ph = rng.uniform(0.0, 2.0 * math.pi)
        f += amp * np.cos(2.0 * math.pi * (kx * X / Lx + ky * Y / Ly) + ph)
    fmin, fmax = f.min(), f.max()
    if fmax - fmin <= 0.0:
        return np.full((ny, nx), 0.5 * (lo + hi))
    return lo + (hi - lo) * (f - fmin) / (fmax - fmin)


@dataclasses.dataclass
class VortexSet:
    centres: np.ndarray   # [k][2] m
    radii: np.ndarray     # [k] m
    signs: np.ndarray     # [k]
    velocities: np.ndarray  # [k][2] m/s (drift of the centres)


def make_vortices(seed: int, Lx: float, Ly: float, n_vortex: int = 3,
                  drift_speed: float = 10.0) -> VortexSet:
    rng = np.random.default_rng(seed)
    c = np.stack([rng.uniform(0.2 * Lx, 0.8 * Lx, n_vortex),
                  rng.uniform(0.2 * Ly, 0.8 * Ly, n_vortex)], axis=1)
    r = rng.uniform(60e3, 120e3, n_vortex)
    s = rng.choice([-1.0, 1.0], n_vortex)
    ang = rng.uniform(0.0, 2.0 * math.pi, n_vortex)
    u = drift_speed * np.stack([np.cos(ang), np.sin(ang)], axis=1)
    return VortexSet(c, r, s, u)


def _reflect(p: float, lo: float, hi: float) -> float:
    span = hi - lo
    q = (p - lo) % (2.0 * span)
    return lo + (q if q <= span else 2.0 * span - q)


def vortex_centres_at(vs: VortexSet, t: float, Lx: float, Ly: float) -> np.ndarray:
    """Centres drifted for time t [s], reflected inside [0.1 L, 0.9 L]."""
    out = np.empty_like(vs.centres)
    for k in range(vs.centres.shape[0]):
        p = vs.centres[k] + vs.velocities[k] * t
        out[k, 0] = _reflect(p[0], 0.1 * Lx, 0.9 * Lx)
        out[k, 1] = _reflect(p[1], 0.1 * Ly, 0.9 * Ly)
    return out


def vortex_wind(vs: VortexSet, nx: int, ny: int, Lx: float, Ly: float,
                vmax: float, t: float = 0.0, inflow_deg: float = 72.0) -> np.ndarray:
    """Sum of Gaussian-shaped rotating vortices at the nodes, rescaled so the
    largest nodal wind speed equals vmax [m/s]."""
    X, Y = node_coords(nx, ny, Lx, Ly)
    a = math.radians(inflow_deg)
    ca, sa = math.cos(a), math.sin(a)
    cen = vortex_centres_at(vs, t, Lx, Ly)
    w = np.zeros((ny + 1, nx + 1, 2))
    for k in range(cen.shape[0]):
        dx, dy = X - cen[k, 0], Y - cen[k, 1]
        R = vs.radii[k]
        g = vs.signs[k] * np.exp(-(dx * dx + dy * dy) / (2.0 * R * R)) / R
        w[..., 0] += g * (ca * dx + sa * dy)
        w[..., 1] += g * (-sa * dx + ca * dy)
    sp = np.sqrt((w ** 2).sum(-1)).max()
    if sp > 0.0:
        w *= vmax / sp
    return w


def ocean_gyre(nx: int, ny: int, Lx: float, Ly: float, vmax: float = 0.1) -> np.ndarray:
    """Rotating gyre of the shape used in Problem II, scaled to vmax [m/s]."""
    X, Y = node_coords(nx, ny, Lx, Ly)
    w = np.empty((ny + 1, nx + 1, 2))
    w[..., 0] = vmax * (-1.0 + 2.0 * Y / Ly)
    w[..., 1] = vmax * (1.0 - 2.0 * X / Lx)
    return w


@dataclasses.dataclass
class Workload:
    name: str
    desc: ProblemDesc
    H: np.ndarray
    A: np.ndarray
    v_air: np.ndarray
    v_ocean: np.ndarray
    v_prev: np.ndarray
    vortices: VortexSet | None = None
    wind_max: float = 15.0

    def fields(self):
        return dict(H=self.H, A=self.A, v_air=self.v_air,
                    v_ocean=self.v_ocean, v_prev=self.v_prev)


def synthetic(n: int, seed: int, h_range=(0.1, 2.0), a_range=(0.7, 1.0),
              wind_max: float = 15.0, delta_min: float = 2e-9, t: float = 0.0,
              name: str = "synthetic", f_coriolis: float = 1.46e-4, ny: int | None = None,
              Ly: float | None = None, order: int = 1) -> Workload:
    """Seeded workload on an n x ny mesh (ny defaults to n) of a 512 km x Ly domain;
    node fields on the nodes of Q1 (order 1) or Q2 (order 2) velocity elements."""
    nx = n
    ny = n if ny is None else ny
    desc = ProblemDesc(nx=nx, ny=ny, delta_min=delta_min, f_coriolis=f_coriolis, order=order)
    if Ly is not None:
        desc = desc.replace(Ly=Ly)
    H = smooth_field(seed, nx, ny, desc.Lx, desc.Ly, *h_range)
    A = smooth_field(seed + 1000, nx, ny, desc.Lx, desc.Ly, *a_range)
    vs = make_vortices(seed + 2000, desc.Lx, desc.Ly)
    va = vortex_wind(vs, order * nx, order * ny, desc.Lx, desc.Ly, wind_max, t)
    vo = ocean_gyre(order * nx, order * ny, desc.Lx, desc.Ly, 0.1)
    vp = np.zeros((order * ny + 1, order * nx + 1, 2))
    return Workload(name, desc, H, A, va, vo, vp, vs, wind_max)


def small_step(n: int = 64) -> Workload:
    """64x64 mesh, seed 1: the small single-step workload (~8.4k unknowns)."""
    return synthetic(n, 1, (0.1, 2.0), (0.7, 1.0), 15.0, 2e-9, name=f"vp_step_{n}")


def medium_steps(n: int = 512) -> Workload:
    """512x512 mesh, seed 2: the multi-step workload (vortices drift 10 m/s)."""
    return synthetic(n, 2, (0.1, 2.0), (0.7, 1.0), 15.0, 2e-9, name=f"vp_steps_{n}")


def sharp_step(n: int = 2048) -> Workload:
    """2048x2048 mesh, seed 3, sharper localisation: wind to 25 m/s,
    H in [0.05, 1.5] m, delta_min = 2e-10 (~8.4M unknowns)."""
    return synthetic(n, 3, (0.05, 1.5), (0.7, 1.0), 25.0, 2e-10, name=f"vp_sharp_{n}")


def advance_wind(w: Workload, t: float) -> np.ndarray:
    """Wind of workload w at time t [s] (vortices drifting)."""
    d = w.desc
    return vortex_wind(w.vortices, d.nx, d.ny, d.Lx, d.Ly, w.wind_max, t)


def sequence_wind(w: Workload, k: int) -> np.ndarray:
    """Wind of step k >= 1 of a workload's sequence: the vortices drifted for (k - 1) dt."""
    return w.v_air if k == 1 else advance_wind(w, (k - 1) * w.desc.dt)


def sequence_step(w: Workload, k: int, v_prev: np.ndarray) -> Workload:
    """Step k >= 1 of a workload's sequence of implicit steps: the same thickness,
    concentration and ocean, the vortices drifted for (k - 1) dt (so step 1 is the
    workload itself), and the previous step's velocity as v_prev."""
    va = sequence_wind(w, k)
    return dataclasses.replace(w, name=f"{w.name}_step{k}", v_air=va,
                               v_prev=np.asarray(v_prev, float).reshape(w.v_prev.shape))


def long_run(n: int = 1024) -> Workload:
    """1024x1024 mesh, seed 5: the 48-step (one day) workload, wind to 25 m/s."""
    return synthetic(n, 5, (0.1, 2.0), (0.7, 1.0), 25.0, 2e-9, name=f"vp_day_{n}")


def problem_one(n: int = 512, order: int = 1) -> Workload:
    """The paper's Problem I (Sec. 5.2): analytic A, H = 2A, constant wind
    (5, 5) m/s, no ocean current, zero Coriolis, delta_min = 2e-9.
    r_1 is taken as printed (its last term is not squared)."""
    desc = ProblemDesc(nx=n, ny=n, f_coriolis=0.0, delta_min=2e-9, order=order)
    X, Y = cell_centres(n, n, desc.Lx, desc.Ly)
    xk, yk = X / 1e6, Y / 1e6  # in units of 1000 km
    r = 0.04 - (xk - 0.25) ** 2 - (yk - 0.25) ** 2
    r1 = 0.1 + (2.0 * xk) ** 2 - 2.0 * yk
    A = 1.0 - 0.5 * np.exp(-800.0 * np.abs(r)) - 0.4 * np.exp(-90.0 * np.abs(r1)) \
        - 0.4 * np.exp(-90.0 * np.abs(r1 + 0.7))
    H = 2.0 * A
    m = order * n + 1
    va = np.zeros((m, m, 2))
    va[..., 0] = 5.0
    va[..., 1] = 5.0
    vo = np.zeros((m, m, 2))
    return Workload(f"problem_one_{n}" + ("_q2" if order == 2 else ""), desc, H, A, va, vo, np.zeros_like(vo),
                    None, 5.0)


DAY = 86400.0


def problem_two_wind(n: int, t: float, Lx: float = 512e3, Ly: float = 512e3) -> np.ndarray:
    """Atmospheric wind of the paper's Problem II (Sec. 5.3) at time t [s]: a
    cyclone whose centre moves along the diagonal at 51.2 km/day (out for 4 days,
    then back), peak factor 15 m/s with the tanh ramps, inflow angle 72 degrees
    (81 after day 4), shape exp(-r/100 km)/50 times the offset in km."""
    td = t / DAY
    if td <= 4.0:
        vmax = -15.0 * math.tanh((4.0 - td) * (4.0 + td) / 2.0)
        alpha = math.radians(72.0)
        m = 256e3 + 51.2e3 * td
    else:
        vmax = 15.0 * math.tanh((12.0 - td) * (-4.0 + td) / 2.0)
        alpha = math.radians(81.0)
        m = 665.6e3 - 51.2e3 * td
    X, Y = node_coords(n, n, Lx, Ly)
    dxk, dyk = (X - m) / 1e3, (Y - m) / 1e3          # offsets in km
    omega = np.exp(-np.sqrt(dxk * dxk + dyk * dyk) / 100.0) / 50.0
    ca, sa = math.cos(alpha), math.sin(alpha)
    w = np.empty((n + 1, n + 1, 2))
    w[..., 0] = omega * vmax * (ca * dxk + sa * dyk)
    w[..., 1] = omega * vmax * (-sa * dxk + ca * dyk)
    return w


def problem_two(n: int = 128, delta_min: float = 2e-9, order: int = 1) -> Workload:
    """Initial state and forcing of the paper's Problem II (Sec. 5.3), the
    time-dependent benchmark: A = 1, H = 0.3 m + 0.005 m (sin(60 x/1000 km) +
    sin(30 y/1000 km)), v = 0, ocean gyre of 0.01 m/s, the moving cyclone at t = 0,
    no Coriolis term (Table tab:params)."""
    desc = ProblemDesc(nx=n, ny=n, f_coriolis=0.0, delta_min=delta_min, order=order)
    X, Y = cell_centres(n, n, desc.Lx, desc.Ly)
    H = 0.3 + 0.005 * (np.sin(60.0 * X / 1e6) + np.sin(30.0 * Y / 1e6))
    A = np.ones((n, n))
    va = problem_two_wind(order * n, 0.0, desc.Lx, desc.Ly)
    vo = ocean_gyre(order * n, order * n, desc.Lx, desc.Ly, 0.01)
    m = order * n + 1
    return Workload(f"problem_two_{n}" + ("_q2" if order == 2 else ""), desc, H, A, va, vo, np.zeros((m, m, 2)),
                    None, 15.0)
