"""Pins of the oracle's fixed-point cloud-in-cell deposit (Sec. IV-A), CPU only."""
from fractions import Fraction

import numpy as np
import pytest

from paper_2010_11540_amd import inputs

ONE = 1 << 24


def _parts(x, y):
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    n = x.shape[0]
    return {"x": x.copy(), "px": np.zeros(n), "y": y.copy(), "py": np.zeros(n),
            "lost": np.zeros(n, dtype=np.uint8)}


@pytest.mark.parametrize("nx,ny", [(64, 64), (128, 128), (40, 24)])
def test_total_charge_is_exactly_conserved(orc, nx, ny):
    g = inputs.make_grid(nx, ny, 4.5e-3, 3.0e-3)
    p = inputs.gaussian_beam(20000, 21, sigma_x=1.5e-3, sigma_y=1.2e-3)
    q, n_in = orc.deposit(p, g)
    assert 0 < n_in < 20000  # some particles fall outside this narrow grid
    assert int(q.sum()) == ONE * n_in
    assert int((p["lost"] == 0).sum()) == n_in
    assert q.min() >= 0


def test_particle_on_a_node_puts_all_charge_there(orc):
    g = inputs.make_grid(16)
    i, j = 5, 9
    x = g["x_min"] + i * g["dx"]
    y = g["y_min"] + j * g["dy"]
    q, n_in = orc.deposit(_parts([x], [y]), g)
    q = q.reshape(16, 16)
    assert n_in == 1
    assert q[i, j] == ONE
    assert q.sum() == ONE


def test_particle_at_cell_centre_splits_in_four(orc):
    g = inputs.make_grid(16)
    x = g["x_min"] + 3.5 * g["dx"]
    y = g["y_min"] + 7.5 * g["dy"]
    q, _ = orc.deposit(_parts([x], [y]), g)
    q = q.reshape(16, 16)
    for a in (3, 4):
        for b in (7, 8):
            assert q[a, b] == ONE // 4


def test_weights_are_the_papers_bilinear_fractions_to_12_bits(orc):
    """Brute force with exact rational arithmetic: each node receives the
    paper's (x_{i+1}-x)(y_{j+1}-y)/(dx dy)-type fraction, quantised per axis to
    1/4096, so the per-node error is below 2 * 2^-13."""
    g = inputs.make_grid(8, 8, 1.0, 1.0)
    rng = np.random.default_rng(9)
    for _ in range(200):
        x = float(rng.uniform(-1.0, 1.0 - 1e-9))
        y = float(rng.uniform(-1.0, 1.0 - 1e-9))
        q, n_in = orc.deposit(_parts([x], [y]), g)
        assert n_in == 1
        q = q.reshape(8, 8)
        fx = (Fraction(x) - Fraction(g["x_min"])) / Fraction(g["dx"])
        fy = (Fraction(y) - Fraction(g["y_min"])) / Fraction(g["dy"])
        i, j = int(fx), int(fy)
        tx, ty = fx - i, fy - j
        exact = {(i, j): (1 - tx) * (1 - ty), (i + 1, j): tx * (1 - ty),
                 (i, j + 1): (1 - tx) * ty, (i + 1, j + 1): tx * ty}
        for (a, b), w in exact.items():
            assert abs(float(Fraction(int(q[a, b]), ONE) - w)) <= 2.0 ** -12 + 1e-15
        nz = {(int(a), int(b)) for a, b in zip(*np.nonzero(q))}
        assert nz <= set(exact)


def test_first_moment_matches_particle_positions(orc):
    """Bilinear assignment preserves the centroid up to the 12-bit quantisation."""
    g = inputs.make_grid(32)
    p = inputs.gaussian_beam(5000, 22)
    q, _ = orc.deposit(p, g)
    q = q.reshape(32, 32).astype(np.float64)
    xs = g["x_min"] + np.arange(32) * g["dx"]
    ys = g["y_min"] + np.arange(32) * g["dy"]
    alive = p["lost"] == 0
    cx = (q.sum(axis=1) * xs).sum() / q.sum()
    cy = (q.sum(axis=0) * ys).sum() / q.sum()
    assert abs(cx - p["x"][alive].mean()) <= g["dx"] / 8192
    assert abs(cy - p["y"][alive].mean()) <= g["dy"] / 8192


def test_permutation_invariance_is_bit_exact(orc):
    g = inputs.make_grid(64)
    p = inputs.gaussian_beam(30000, 23)
    perm = np.random.default_rng(1).permutation(30000)
    p2 = {k: v[perm].copy() for k, v in p.items()}
    q1, n1 = orc.deposit(p, g)
    q2, n2 = orc.deposit(p2, g)
    assert n1 == n2
    np.testing.assert_array_equal(q1, q2)


def test_domain_edges_nan_and_inf(orc):
    g = inputs.make_grid(16)
    top = g["x_min"] + 15 * g["dx"]
    xs = [g["x_min"], top, top - 1e-6 * g["dx"], np.nan, 0.0, np.inf, -np.inf, 0.0]
    ys = [0.0, 0.0, 0.0, 0.0, np.nan, 0.0, 0.0, g["y_min"] - 1e-12]
    p = _parts(xs, ys)
    q, n_in = orc.deposit(p, g)
    np.testing.assert_array_equal(p["lost"], [0, 1, 0, 1, 1, 1, 1, 1])
    assert n_in == 2
    assert int(q.sum()) == 2 * ONE


def test_all_particles_on_one_node(orc):
    """Adversarial clustering: 2^16 particles on one node -> 2^40 units."""
    g = inputs.make_grid(16)
    n = 1 << 16
    x = np.full(n, g["x_min"] + 7 * g["dx"])
    y = np.full(n, g["y_min"] + 2 * g["dy"])
    q, n_in = orc.deposit(_parts(x, y), g)
    assert n_in == n
    assert q.reshape(16, 16)[7, 2] == n * ONE


def test_lost_particles_do_not_deposit(orc):
    g = inputs.make_grid(32)
    p = inputs.gaussian_beam(1000, 24)
    p["lost"][:500] = 1
    q, n_in = orc.deposit(p, g)
    q2, n2 = orc.deposit({k: v[500:].copy() for k, v in p.items()}, g)
    assert n_in == n2
    np.testing.assert_array_equal(q, q2)
