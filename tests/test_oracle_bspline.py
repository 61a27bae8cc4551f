"""Pins of the oracle's potential interpolation (Sec. IV-C, read as the
uniform bicubic B-spline with the node potentials as control points; the
printed Bezier form jumps across cells) and its analytic-gradient field:

  * a linear potential gives exactly its value and constant field;
  * potentials varying in one axis only, or separable, match scipy's cubic
    BSpline with the same uniform knots (value and derivative);
  * the field is continuous across cell edges (C1) and so is its derivative (C2);
  * the field of a round Gaussian beam's analytic potential converges at
    second order in the grid spacing.
"""
import numpy as np
import pytest
from scipy.interpolate import BSpline
from scipy.special import exp1

from paper_2010_11540_amd import inputs


def _nodes(grid):
    xs = grid["x_min"] + grid["dx"] * np.arange(-1, grid["nx"] + 1)
    ys = grid["y_min"] + grid["dy"] * np.arange(-1, grid["ny"] + 1)
    return xs, ys


def _points(grid, n, seed, margin=0.0):
    rng = np.random.default_rng(seed)
    lx = (grid["nx"] - 1) * grid["dx"]
    ly = (grid["ny"] - 1) * grid["dy"]
    x = grid["x_min"] + margin + rng.random(n) * (lx - 2 * margin)
    y = grid["y_min"] + margin + rng.random(n) * (ly - 2 * margin)
    return x, y


def test_linear_potential_exact(orc):
    grid = inputs.make_grid(32, 16, 5e-3, 3e-3)
    xs, ys = _nodes(grid)
    a, b, c = 3.7, -2.2, 0.4
    phi = a * xs[:, None] + b * ys[None, :] + c
    x, y = _points(grid, 5000, 1)
    u, ex, ey = orc.bspline_eval(x, y, phi, grid)
    np.testing.assert_allclose(u, a * x + b * y + c, rtol=0, atol=1e-14)
    np.testing.assert_allclose(ex, -a, rtol=1e-12)
    np.testing.assert_allclose(ey, -b, rtol=1e-12)


def _scipy_spline(nodes, values, h):
    # cubic basis centred on each node: knots one spacing apart, three before
    # the first node centre
    t = nodes[0] + h * (np.arange(len(values) + 4) - 2)
    return BSpline(t, values, 3)


def test_one_axis_and_separable_match_scipy(orc):
    grid = inputs.make_grid(16, 32, 4e-3, 6e-3)
    xs, ys = _nodes(grid)
    rng = np.random.default_rng(3)
    f, g = rng.normal(size=xs.size), rng.normal(size=ys.size)
    sf, sg = _scipy_spline(xs, f, grid["dx"]), _scipy_spline(ys, g, grid["dy"])
    x, y = _points(grid, 3000, 4)
    u, ex, ey = orc.bspline_eval(x, y, f[:, None] * np.ones_like(ys)[None, :], grid)
    np.testing.assert_allclose(u, sf(x), rtol=0, atol=1e-13)
    np.testing.assert_allclose(ex, -sf.derivative()(x), rtol=0, atol=1e-9)
    np.testing.assert_allclose(ey, 0.0, atol=1e-9)
    u, ex, ey = orc.bspline_eval(x, y, f[:, None] * g[None, :], grid)
    np.testing.assert_allclose(u, sf(x) * sg(y), rtol=0, atol=1e-13)
    np.testing.assert_allclose(ex, -sf.derivative()(x) * sg(y), rtol=0, atol=1e-9)
    np.testing.assert_allclose(ey, -sf(x) * sg.derivative()(y), rtol=0, atol=1e-9)


def test_field_and_its_derivative_continuous_across_cells(orc):
    grid = inputs.make_grid(16)
    xs, ys = _nodes(grid)
    phi = np.random.default_rng(7).normal(size=(xs.size, ys.size))
    eps = 1e-9 * grid["dx"]
    yv = grid["y_min"] + 6.3 * grid["dy"]
    for i in range(1, grid["nx"] - 1):
        xi = grid["x_min"] + i * grid["dx"]
        x = np.array([xi - eps, xi + eps, xi - 2 * eps, xi + 2 * eps])
        u, ex, ey = orc.bspline_eval(x, np.full(4, yv), phi, grid)
        assert abs(ex[0] - ex[1]) < 1e-6 * np.abs(ex).max() + 1e-12
        assert abs(ey[0] - ey[1]) < 1e-6 * np.abs(ey).max() + 1e-12
        # second derivative from one-sided differences on each side
        d_left = (ex[0] - ex[2]) / eps
        d_right = (ex[3] - ex[1]) / eps
        assert abs(d_left - d_right) < 1e-3 * max(abs(d_left), 1.0 / grid["dx"] ** 2 * 1e-9)


@pytest.mark.parametrize("n", [32, 64, 128])
def test_round_gaussian_field_converges(orc, n):
    """phi(r) = -(ln(r^2/2s^2) + E1(r^2/2s^2))/2 (a unit line charge with a
    Gaussian profile, E_r = (1 - exp(-r^2/2s^2))/r); the B-spline surface's
    smoothing error is O(h^2): the error at 2n is about a quarter of that at n."""
    s = 1e-3

    def err(nn):
        grid = inputs.make_grid(nn)
        xs, ys = _nodes(grid)
        r2 = xs[:, None] ** 2 + ys[None, :] ** 2
        q = r2 / (2 * s * s)
        phi = -0.5 * (np.log(q) + exp1(q))
        x, y = _points(grid, 4000, 11, margin=2e-3)
        rr = np.hypot(x, y)
        keep = rr > 0.5 * s
        _, ex, ey = orc.bspline_eval(x[keep], y[keep], phi, grid)
        er = (1 - np.exp(-rr[keep] ** 2 / (2 * s * s))) / rr[keep]
        return max(np.abs(ex - er * x[keep] / rr[keep]).max(),
                   np.abs(ey - er * y[keep] / rr[keep]).max()) / er.max()

    e1, e2 = err(n), err(2 * n)
    assert 3.0 < e1 / e2 < 5.0, (e1, e2)
