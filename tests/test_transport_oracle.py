"""Pins of the transport oracle (explicit upwind finite volumes for A and H)."""
import numpy as np

from oracle import transport as T


def _field(rng, nx, ny, lo, hi):
    return lo + (hi - lo) * rng.random((ny, nx))


def _vel(rng, nx, ny, scale):
    v = scale * rng.standard_normal((ny + 1, nx + 1, 2))
    v[0], v[-1], v[:, 0], v[:, -1] = 0.0, 0.0, 0.0, 0.0     # zero Dirichlet velocity
    return v.ravel()


def test_conservation_without_clipping():
    """With no flux through the boundary the cell sums of A and H are unchanged."""
    rng = np.random.default_rng(0)
    nx, ny, L = 23, 17, 512e3
    A, H = _field(rng, nx, ny, 0.2, 1.0), _field(rng, nx, ny, 0.1, 2.0)
    v = _vel(rng, nx, ny, 0.1)
    A1, H1 = T.advect(v, A, H, nx, ny, L, L * ny / nx, 1800.0, clip=False)
    assert abs(A1.sum() - A.sum()) < 1e-12 * A.sum()
    assert abs(H1.sum() - H.sum()) < 1e-12 * H.sum()
    assert np.abs(A1 - A).max() > 1e-6          # something moved


def test_uniform_shift_is_the_upwind_stencil():
    """Uniform flow u > 0 in x: interior cells get Q_i - c (Q_i - Q_{i-1}),
    c = u dt / hx (the first-order upwind scheme in closed form)."""
    nx, ny, L, u, dt = 20, 6, 512e3, 0.2, 1800.0
    hx = L / nx
    v = np.zeros((ny + 1, nx + 1, 2))
    v[1:-1, 1:-1, 0] = u                        # nodal u; faces of interior rows see u or u/2
    rng = np.random.default_rng(1)
    H = _field(rng, nx, ny, 0.1, 2.0)
    A = np.ones((ny, nx))
    A1, H1 = T.advect(v.ravel(), A, H, nx, ny, L, 0.37 * L, dt, clip=False)   # hy != hx
    c = u * dt / hx
    j = slice(2, ny - 2)                        # rows whose faces all carry exactly u
    ref = H[j, 2:-2] - c * (H[j, 2:-2] - H[j, 1:-3])
    assert np.allclose(H1[j, 2:-2], ref, rtol=0, atol=1e-14)
    # constant A in a divergence-free interior stays constant
    assert np.allclose(A1[j, 2:-2], 1.0, atol=1e-14)


def test_reversed_flow_uses_the_other_neighbour():
    nx, ny, L, u, dt = 20, 6, 512e3, -0.2, 1800.0
    hx = L / nx
    v = np.zeros((ny + 1, nx + 1, 2))
    v[1:-1, 1:-1, 0] = u
    rng = np.random.default_rng(2)
    H = _field(rng, nx, ny, 0.1, 2.0)
    _, H1 = T.advect(v.ravel(), np.ones((ny, nx)), H, nx, ny, L, 0.37 * L, dt, clip=False)
    c = -u * dt / hx
    j = slice(2, ny - 2)
    ref = H[j, 2:-2] - c * (H[j, 2:-2] - H[j, 3:-1])
    assert np.allclose(H1[j, 2:-2], ref, rtol=0, atol=1e-14)


def test_uniform_shift_in_y():
    """Uniform flow in y on cells with hy != hx: Q_j - (w dt / hy) (Q_j - Q_{j-1})."""
    nx, ny, L, w, dt = 7, 18, 512e3, 0.15, 1800.0
    Ly = 0.6 * L
    hy = Ly / ny
    v = np.zeros((ny + 1, nx + 1, 2))
    v[1:-1, 1:-1, 1] = w
    rng = np.random.default_rng(5)
    H = _field(rng, nx, ny, 0.1, 2.0)
    _, H1 = T.advect(v.ravel(), np.ones((ny, nx)), H, nx, ny, L, Ly, dt, clip=False)
    c = w * dt / hy
    i = slice(2, nx - 2)
    ref = H[2:-2, i] - c * (H[2:-2, i] - H[1:-3, i])
    assert np.allclose(H1[2:-2, i], ref, rtol=0, atol=1e-14)


def test_transposed_problem_gives_transposed_result():
    """Swapping x and y (fields transposed, velocity components swapped) transposes
    the result: catches an exchanged face orientation or spacing."""
    rng = np.random.default_rng(3)
    nx, ny, L = 13, 9, 512e3
    Ly = L * ny / nx
    A, H = _field(rng, nx, ny, 0.2, 1.0), _field(rng, nx, ny, 0.1, 2.0)
    v = _vel(rng, nx, ny, 0.2).reshape(ny + 1, nx + 1, 2)
    A1, H1 = T.advect(v.ravel(), A, H, nx, ny, L, Ly, 1800.0, clip=False)
    vt = np.ascontiguousarray(v.transpose(1, 0, 2)[..., ::-1])
    A2, H2 = T.advect(vt.ravel(), A.T, H.T, ny, nx, Ly, L, 1800.0, clip=False)
    assert np.allclose(A2, A1.T, rtol=0, atol=1e-13)
    assert np.allclose(H2, H1.T, rtol=0, atol=1e-13)


def test_clipping_bounds():
    rng = np.random.default_rng(4)
    nx, ny, L = 16, 16, 512e3
    A, H = np.ones((ny, nx)), _field(rng, nx, ny, 0.0, 0.05)
    v = _vel(rng, nx, ny, 1.0)
    A1, H1 = T.advect(v, A, H, nx, ny, L, L, 1800.0)
    assert A1.max() <= 1.0 and A1.min() >= 0.0 and H1.min() >= 0.0


def test_q2_face_means_are_exact_for_quadratic_traces():
    """With Q2 velocity the face mean uses the face's end and midpoint values and is
    the exact mean of a quadratic trace: u = (1 + y/Ly)^2 on vertical faces."""
    nx, ny, Lx, Ly = 5, 4, 512e3, 300e3
    X, Y = np.meshgrid(np.linspace(0, Lx, 2 * nx + 1), np.linspace(0, Ly, 2 * ny + 1), indexing="xy")
    v = np.stack([(1 + Y / Ly) ** 2, (2 - X / Lx) ** 2], -1)
    ux, uy = T.face_velocities(v.ravel(), nx, ny, order=2)
    hy, hx = Ly / ny, Lx / nx
    for j in range(ny):
        y0, y1 = j * hy, (j + 1) * hy
        exact = ((1 + y1 / Ly) ** 3 - (1 + y0 / Ly) ** 3) * Ly / 3 / hy
        assert np.allclose(ux[j, 1:-1], exact, rtol=1e-13)
    for i in range(nx):
        x0, x1 = i * hx, (i + 1) * hx
        exact = -((2 - x1 / Lx) ** 3 - (2 - x0 / Lx) ** 3) * Lx / 3 / hx
        assert np.allclose(uy[1:-1, i], exact, rtol=1e-13)
    assert np.all(ux[:, [0, -1]] == 0.0) and np.all(uy[[0, -1], :] == 0.0)
