"""Pins of the oracle's long-bunch space-charge step (Sec. IV): the line
density lambda(sigma) as a one-dimensional fixed-point histogram, the
transverse kick scaled by lambda/lambda_peak and the longitudinal kick
-gamma0 kappa phi lambda'/lambda_peak with the grounded-pipe potential.

Pinned against: exact integer conservation and node cases; the histogram's
centroid; the closed-form Gaussian and its derivative; the already pinned
transverse pipe step (a flat bunch must reproduce it bit for bit in its
interior and give no longitudinal kick there); the signs of the longitudinal
kick of a Gaussian bunch in a grounded pipe.
"""
import math

import numpy as np
import pytest
from scipy.special import ndtri

from paper_2010_11540_amd import inputs

FRAC = 4096


def _beam(n, seed, sig):
    b = inputs.gaussian_beam6d(n, seed, 1e-3, 1e-3, 1e-3, 1e-3)
    b["sigma"] = np.ascontiguousarray(sig, dtype=np.float64)
    return b


def test_line_histogram_conserves_and_marks_lost(orc):
    line = inputs.make_line(3.0, 64)
    grid = inputs.make_grid(32)
    rng = np.random.default_rng(5)
    sig = rng.normal(0, 1.2, 20_000)
    sig[:5] = [np.nan, np.inf, -3.0 - 1e-9, 3.0, line["z_min"] + 17 * line["dz"]]
    b = _beam(sig.size, 6, sig)
    q, h, n_in = orc.deposit_line(b, grid, line)
    out = ~((sig >= -3.0) & (sig < -3.0 + 63 * line["dz"]))
    tr_out = ~((np.abs(b["x"]) < 6e-3) & (np.abs(b["y"]) < 6e-3))
    assert n_in == np.count_nonzero(~(out | (b["lost"].astype(bool) & ~out)))
    assert h.sum() == FRAC * n_in and q.sum() == FRAC * FRAC * n_in
    assert b["lost"][:4].all() and not b["lost"][4]
    # every lost particle is outside one of the two domains
    lost = b["lost"].astype(bool)
    assert np.all(out[lost] | tr_out[lost])
    # a particle exactly on node 17 puts all its weight there
    one = _beam(1, 1, [line["z_min"] + 17 * line["dz"]])
    one["x"][:] = 0.0
    one["y"][:] = 0.0
    _, h1, _ = orc.deposit_line(one, grid, line)
    assert h1[17] == FRAC and h1.sum() == FRAC


def test_line_histogram_centroid(orc):
    line = inputs.make_line(4.0, 128)
    rng = np.random.default_rng(8)
    sig = rng.normal(0.3, 0.8, 50_000)
    b = _beam(sig.size, 9, sig)
    b["x"][:] = 0.0
    b["y"][:] = 0.0
    _, h, n_in = orc.deposit_line(b, inputs.make_grid(16), line)
    z = line["z_min"] + line["dz"] * np.arange(line["nz"])
    inside = b["lost"] == 0
    cen = (h * z).sum() / h.sum()
    # each particle's weight is rounded to 1/4096 of a cell: |shift| <= dz/8192
    assert abs(cen - sig[inside].mean()) <= line["dz"] / 8192 + 1e-15


def test_line_table_of_a_gaussian(orc):
    """Quantiles of a unit Gaussian (no sampling noise) on 128 nodes over
    +-6: lambda/lambda_peak and lambda'/lambda_peak against exp(-z^2/2) and
    -z exp(-z^2/2), within the cloud-in-cell and centred-difference
    discretisation (dz^2 terms)."""
    n = 400_000
    sig = ndtri((np.arange(n) + 0.5) / n)
    line = inputs.make_line(6.0, 128)
    b = _beam(n, 2, sig)
    b["x"][:] = 0.0
    b["y"][:] = 0.0
    _, h, _ = orc.deposit_line(b, inputs.make_grid(16), line)
    lw, ld = orc.line_table(h, line)
    z = line["z_min"] + line["dz"] * np.arange(line["nz"])
    peak = h.max() / (FRAC * n * line["dz"]) * math.sqrt(2 * math.pi)  # lambda_peak / lambda(0)
    assert np.abs(lw * peak - np.exp(-z * z / 2)).max() < 3e-3
    assert np.abs(ld * peak - (-z * np.exp(-z * z / 2))).max() < 5e-3
    assert lw.max() == 1.0


def _flat_bunch(line, per_cell=24, n_cells=80, first=24):
    """sigma at the same fractions of every cell from node `first` on: the
    histogram is exactly constant on the interior nodes."""
    f = (np.arange(per_cell) + 0.37) / per_cell
    k = first + np.arange(n_cells)
    return (line["z_min"] + (k[:, None] + f[None, :]) * line["dz"]).ravel()


def test_flat_bunch_reproduces_the_transverse_pipe_step(orc):
    line = inputs.make_line(6.0, 128)
    sig = _flat_bunch(line)
    n = sig.size
    grid = inputs.make_grid(64)
    base = _beam(n, 31, sig)
    scale = 1.0 / ((1 << 24) * n)
    a = inputs.copy_parts(base)
    lw, ld, _, n_in = orc.space_charge_line(a, grid, line, scale, 3e-7)
    assert n_in == n
    ref = inputs.copy_parts(base)
    orc.space_charge(ref, grid, scale, 3e-7, solver="pipe")
    k = np.floor((sig - line["z_min"]) / line["dz"]).astype(int)
    interior = (k >= 26) & (k <= 24 + 80 - 3)
    assert np.all(lw[27:24 + 80 - 1] == 1.0) and np.all(ld[27:24 + 80 - 2] == 0.0)
    for c in ("x", "px", "y", "py"):
        np.testing.assert_array_equal(a[c][interior], ref[c][interior])
    np.testing.assert_array_equal(a["psigma"][interior], base["psigma"][interior])
    assert np.any(a["psigma"][~interior] != base["psigma"][~interior])


def test_gaussian_bunch_longitudinal_kick_signs_and_probe(orc):
    """In a grounded pipe the potential of a positive beam is positive
    inside, so the kick -gamma0 kappa phi lambda'/lambda_peak pushes the head
    (sigma > 0, lambda' < 0) forward and the tail back.  A probe on a
    transverse node and a line node takes exactly the node values."""
    n = 100_000
    rng = np.random.default_rng(12)
    sig = rng.permutation(ndtri((np.arange(n) + 0.5) / n))  # smooth line density
    line = inputs.make_line(6.0, 128)
    grid = inputs.make_grid(64)
    base = _beam(n, 13, sig)
    i0, j0, k0 = 30, 37, 80
    base["x"][0] = grid["x_min"] + i0 * grid["dx"]
    base["y"][0] = grid["y_min"] + j0 * grid["dy"]
    base["sigma"][0] = line["z_min"] + k0 * line["dz"]
    scale, kappa = 1.0 / ((1 << 24) * n), 2e-7
    a = inputs.copy_parts(base)
    lw, ld, phi, _ = orc.space_charge_line(a, grid, line, scale, kappa)
    dps = a["psigma"] - base["psigma"]
    alive = a["lost"] == 0
    assert (phi[2:-1, 2:-1] > 0).all()  # nodes 1..n-1; node 0 and node n are the walls
    head = alive & (sig > 2 * line["dz"]) & (sig < 3.0)
    tail = alive & (sig < -2 * line["dz"]) & (sig > -3.0)
    assert (dps[head] > 0).all() and (dps[tail] < 0).all()
    want = -line["gamma0"] * kappa * phi[i0 + 1, j0 + 1] * ld[k0]
    assert dps[0] == pytest.approx(want, rel=1e-11)  # p_sigma + kick - p_sigma rounds
    ref = inputs.copy_parts(base)
    orc.space_charge(ref, grid, scale, kappa, solver="pipe")
    assert a["px"][0] - base["px"][0] == pytest.approx(lw[k0] * (ref["px"][0] - base["px"][0]),
                                                        rel=1e-14)


def test_off_node_probe_interpolates_potential_and_line(orc):
    """A probe at fractions (1/4, 3/4) of a transverse cell and 1/4 of a line
    cell (exact in the 12-bit weights): its longitudinal kick uses phi and
    lambda'/lambda_peak interpolated bilinearly and linearly from the nodes,
    checked with scipy's grid interpolator and numpy's interp."""
    from scipy.interpolate import RegularGridInterpolator
    n = 60_000
    rng = np.random.default_rng(21)
    sig = rng.permutation(ndtri((np.arange(n) + 0.5) / n))
    line = inputs.make_line(6.0, 128)
    grid = inputs.make_grid(64)
    base = _beam(n, 22, sig)
    i0, j0, k0 = 25, 41, 75
    px_, py_ = grid["x_min"] + (i0 + 0.25) * grid["dx"], grid["y_min"] + (j0 + 0.75) * grid["dy"]
    pz = line["z_min"] + (k0 + 0.25) * line["dz"]
    base["x"][0], base["y"][0], base["sigma"][0] = px_, py_, pz
    scale, kappa = 1.0 / ((1 << 24) * n), 2e-7
    a = inputs.copy_parts(base)
    lw, ld, phi, _ = orc.space_charge_line(a, grid, line, scale, kappa)
    xs = grid["x_min"] + grid["dx"] * np.arange(-1, grid["nx"] + 1)
    ys = grid["y_min"] + grid["dy"] * np.arange(-1, grid["ny"] + 1)
    phi_p = RegularGridInterpolator((xs, ys), phi)([[px_, py_]])[0]
    zs = line["z_min"] + line["dz"] * np.arange(line["nz"])
    d_p = np.interp(pz, zs, ld)
    want = -line["gamma0"] * kappa * phi_p * d_p
    assert a["psigma"][0] - base["psigma"][0] == pytest.approx(want, rel=1e-10)
    w_p = np.interp(pz, zs, lw)
    ref = inputs.copy_parts(base)
    orc.space_charge(ref, grid, scale, kappa, solver="pipe")
    assert a["py"][0] - base["py"][0] == pytest.approx(w_p * (ref["py"][0] - base["py"][0]),
                                                        rel=1e-12)
