"""Pins of the oracle's grounded-pipe solve (Sec. IV-B: the 5-point discrete
Poisson equation with u = 0 on the walls of a rectangular pipe).

The walls pass through node 0 and node n of each axis (node n is one spacing
past the last grid node).  What fixes the answer independently of the
oracle's eigen-expansion: the discrete equation itself (its residual), the
wall values, the symmetry of the pipe, and the open-boundary limit (the
free-space Green's function -ln r, pinned elsewhere by closed forms) for a
beam far from the walls."""
import numpy as np
import pytest

from paper_2010_11540_amd import inputs


def _grid(nx, ny, dx, dy):
    return {"nx": nx, "ny": ny, "x_min": 0.0, "y_min": 0.0, "dx": dx, "dy": dy}


def _random_charge(nx, ny, seed):
    rng = np.random.default_rng(seed)
    return rng.integers(0, 1 << 24, size=nx * ny).astype(np.int64)


@pytest.mark.parametrize("nx,ny,dx,dy", [(32, 16, 1e-4, 2.5e-4), (16, 16, 3e-4, 3e-4),
                                         (8, 64, 2e-4, 1e-4)])
def test_pipe_potential_solves_the_discrete_poisson_equation(orc, nx, ny, dx, dy):
    g = _grid(nx, ny, dx, dy)
    q = _random_charge(nx, ny, nx * ny)
    scale = 1.0 / (1 << 24) / 1000.0
    phi = orc.potential(q, scale, g, "pipe")  # nodes -1..nx, -1..ny
    c = phi[1:-1, 1:-1]  # nodes 0..nx-1, 0..ny-1; node nx (the last row) is the wall
    lap = ((phi[2:, 1:-1] - 2 * c + phi[:-2, 1:-1]) / dx ** 2 +
           (phi[1:-1, 2:] - 2 * c + phi[1:-1, :-2]) / dy ** 2)
    f = -2 * np.pi * q.reshape(nx, ny) * scale / (dx * dy)
    res = lap[1:, 1:] - f[1:, 1:]                          # interior nodes
    assert np.abs(res).max() <= 1e-12 * np.abs(f).max(), np.abs(res).max() / np.abs(f).max()


def test_pipe_walls_are_grounded_and_take_the_wall_charge(orc):
    nx, ny = 32, 16
    g = _grid(nx, ny, 1e-4, 2e-4)
    q = _random_charge(nx, ny, 5)
    scale = 1e-9
    phi = orc.potential(q, scale, g, "pipe")
    # node 0 (index 1) and node nx / ny (last index) are the walls
    assert not np.any(phi[1, :]) and not np.any(phi[:, 1])
    assert not np.any(phi[-1, :]) and not np.any(phi[:, -1])
    # node -1 is the odd image of node 1
    np.testing.assert_array_equal(phi[0, 1:-1], -phi[2, 1:-1])
    np.testing.assert_array_equal(phi[1:-1, 0], -phi[1:-1, 2])
    # charge on the wall nodes changes nothing
    q2 = q.reshape(nx, ny).copy()
    q2[0, :] += 12345
    q2[:, 0] += 777
    phi2 = orc.potential(q2.ravel(), scale, g, "pipe")
    np.testing.assert_array_equal(phi, phi2)


def test_pipe_field_is_antisymmetric_about_the_pipe_centre(orc):
    nx, ny = 32, 32
    g = _grid(nx, ny, 1e-4, 1e-4)
    rng = np.random.default_rng(9)
    base = rng.integers(0, 1 << 20, size=(nx // 2 + 1, ny))
    # mirror image about the pipe centre (node nx/2): q[i] = q[nx - i]
    q = np.array([base[min(i, nx - i)] for i in range(nx)], dtype=np.int64)
    ex, ey = orc.solve(q.ravel(), 1e-9, g, "pipe")
    ex = ex.reshape(nx, ny)
    for i in range(1, nx):
        np.testing.assert_allclose(ex[i], -ex[nx - i], rtol=0, atol=1e-12 * np.abs(ex).max())


def test_wide_pipe_field_approaches_the_open_boundary_field(orc):
    """A small round beam in the middle of a pipe 16 beam sigmas across: the
    walls' image charges change the field near the beam by about (r/L)^2 of
    it, L the distance to the walls."""
    n = 128
    d = 1e-4
    g = _grid(n, n, d, d)
    c = (n // 2) * d
    sigma = 4 * d
    parts = inputs.gaussian_beam(200_000, 21, sigma_x=sigma, sigma_y=sigma)
    parts["x"] += c
    parts["y"] += c
    q, n_in = orc.deposit(parts, g)
    scale = 1.0 / ((1 << 24) * n_in)
    ex_o, ey_o = orc.solve(q, scale, g, "open")
    ex_p, ey_p = orc.solve(q, scale, g, "pipe")
    i0 = n // 2
    r = np.hypot(*np.meshgrid((np.arange(n) - i0) * d, (np.arange(n) - i0) * d, indexing="ij"))
    near = (r <= 2 * sigma).ravel()
    e_open = np.hypot(ex_o, ey_o)
    diff = np.hypot(ex_p - ex_o, ey_p - ey_o)
    rel = diff[near].max() / e_open[near].max()
    bound = 4 * (2 * sigma / (i0 * d)) ** 2
    print(f"wide pipe vs open boundary near the beam: {rel:.3e} (bound {bound:.3e})")
    assert rel <= bound
    # and the walls matter: far from the beam the fields differ
    far = (r >= 0.8 * i0 * d).ravel()
    assert diff[far].max() > 0.1 * e_open[far].max()
