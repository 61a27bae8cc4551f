"""Pins of the oracle's thick elements (Sec. III-B chromatic thick quadrupole,
Sec. III-C thick sextupole by the symmetric split of eq. Sym2) to things other
than the oracle's own formulas:

  * Hamilton's equations of H_approx (eq. H with h = 0), built here from the
    Hamiltonian by complex-step differentiation (no hand-derived equations of
    motion) and integrated with an 8th-order Runge-Kutta method to 1e-13;
  * symplecticity of every element's 6x6 Jacobian (J^T Omega J = Omega);
  * the exact flow's group property and the split's time-reversal symmetry;
  * second-order convergence of the split in the step count;
  * the linear limit: at p_sigma = 0 the thick quadrupole is the matrix
    exponential of its linear system.
"""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp
from scipy.linalg import expm

from paper_2010_11540_amd import inputs

IG2 = 1.0 / inputs.GAMMA0_3GEV ** 2
OMEGA = np.zeros((6, 6))
for _k in range(3):
    OMEGA[2 * _k, 2 * _k + 1] = 1.0
    OMEGA[2 * _k + 1, 2 * _k] = -1.0


def h_approx(v, k1, k2, ig2):
    """eq. H, h = 0, with e A_s / p0 = -k1 (x^2 - y^2)/2 - k2 (x^3 - 3 x y^2)/6."""
    x, px, y, py, s, ps = v
    p2 = px * px + py * py
    return (0.5 * p2 + 0.5 * ps * ps * ig2 - 0.5 * p2 * ps
            + 0.5 * k1 * (x * x - y * y) + k2 * (x ** 3 - 3 * x * y * y) / 6.0)


def _rhs(k1, k2, ig2):
    def f(_s, v):
        g = np.empty(6)
        for i in range(6):  # complex-step gradient: exact to rounding for analytic H
            d = np.zeros(6, dtype=complex)
            d[i] = 1e-30j
            g[i] = h_approx(v + d, k1, k2, ig2).imag / 1e-30
        # dq/ds = dH/dp, dp/ds = -dH/dq for the pairs (x,px), (y,py), (sigma,p_sigma)
        return np.array([g[1], -g[0], g[3], -g[2], g[5], -g[4]])
    return f


def integrate(v0, length, k1=0.0, k2=0.0, ig2=IG2):
    r = solve_ivp(_rhs(k1, k2, ig2), (0.0, length), np.asarray(v0, float), method="DOP853",
                  rtol=1e-13, atol=1e-18)
    assert r.success
    return r.y[:, -1]


def push6(orc, v, lattice):
    p = {k: np.array([float(c)]) for k, c in zip(("x", "px", "y", "py", "sigma", "psigma"), v)}
    orc.push(p, lattice)
    return np.array([p[k][0] for k in ("x", "px", "y", "py", "sigma", "psigma")])


def jacobian(orc, v, lattice, h=1e-6):
    v = np.asarray(v, float)
    j = np.empty((6, 6))
    for i in range(6):
        d = np.zeros(6)
        d[i] = h
        j[:, i] = (push6(orc, v + d, lattice) - push6(orc, v - d, lattice)) / (2 * h)
    return j


STATES = [np.array([1.2e-3, -4e-4, -7e-4, 9e-4, 0.3, 2e-3]),
          np.array([-2e-3, 1.1e-3, 1.5e-3, -2e-4, -1.1, -0.04]),
          np.array([3e-3, 0.0, 0.0, 2e-3, 0.0, 0.08])]


@pytest.mark.parametrize("k1", [0.8, -1.3, 0.0, 1e-9])
@pytest.mark.parametrize("state", range(len(STATES)))
def test_thick_quad_is_the_flow_of_h_approx(orc, k1, state):
    v0 = STATES[state]
    length = 0.7
    got = push6(orc, v0, inputs.quad_thick(k1, length, IG2))
    want = integrate(v0, length, k1=k1)
    scale = np.array([1e-3, 1e-3, 1e-3, 1e-3, 1e-3, 1e-3])
    err = np.abs(got - want) / scale
    assert err.max() < 1e-10, (got - want)
    assert got[5] == v0[5]


@pytest.mark.parametrize("k1", [0.8, -1.3])
def test_thick_quad_linear_limit_is_matrix_exponential(orc, k1):
    length = 0.45
    ax = np.array([[0.0, 1.0], [-k1, 0.0]])
    ay = np.array([[0.0, 1.0], [k1, 0.0]])
    mx, my = expm(ax * length), expm(ay * length)
    v0 = np.array([1e-3, 2e-4, -5e-4, 3e-4, 0.2, 0.0])
    got = push6(orc, v0, inputs.quad_thick(k1, length, IG2))
    np.testing.assert_allclose(got[:2], mx @ v0[:2], rtol=0, atol=1e-17)
    np.testing.assert_allclose(got[2:4], my @ v0[2:4], rtol=0, atol=1e-17)


def test_thick_quad_group_property(orc):
    v0 = STATES[1]
    whole = push6(orc, v0, inputs.quad_thick(0.9, 1.0, IG2))
    parts = push6(orc, v0, np.concatenate([inputs.quad_thick(0.9, 0.35, IG2),
                                           inputs.quad_thick(0.9, 0.65, IG2)]))
    np.testing.assert_allclose(parts, whole, rtol=0, atol=1e-15)


@pytest.mark.parametrize("element", ["quad_f", "quad_d", "sext1", "sext4"])
def test_thick_elements_are_symplectic(orc, element):
    lat = {"quad_f": inputs.quad_thick(1.1, 0.6, IG2),
           "quad_d": inputs.quad_thick(-0.7, 0.6, IG2),
           "sext1": inputs.sext_thick(300.0, 0.4, IG2, 1),
           "sext4": inputs.sext_thick(-200.0, 0.4, IG2, 4)}[element]
    j = jacobian(orc, STATES[0], lat)
    np.testing.assert_allclose(j.T @ OMEGA @ j, OMEGA, rtol=0, atol=1e-8)
    assert abs(np.linalg.det(j) - 1.0) < 1e-8


def test_thick_sextupole_without_strength_is_the_exact_drift(orc):
    for v0 in STATES:
        got = push6(orc, v0, inputs.sext_thick(0.0, 1.7, IG2, 1))
        want = integrate(v0, 1.7)
        np.testing.assert_allclose(got, want, rtol=0, atol=1e-14)


def test_thick_sextupole_split_is_time_symmetric(orc):
    v0 = STATES[2]
    fwd = push6(orc, v0, inputs.sext_thick(400.0, 0.5, IG2, 3))
    back = push6(orc, fwd, inputs.sext_thick(400.0, -0.5, IG2, 3))
    np.testing.assert_allclose(back, v0, rtol=0, atol=1e-15)


def test_thick_sextupole_converges_at_second_order(orc):
    """The split's error against the exact flow of H0 + V falls by about 4x
    per halving of the step (error O(h^2) for a second-order symmetric
    method; the SABA2 coefficients make the leading term small but keep it)."""
    v0 = np.array([4e-3, 1e-3, -3e-3, 5e-4, 0.1, 0.02])
    k2, length = 2000.0, 0.5
    want = integrate(v0, length, k2=k2)
    errs = []
    for n in (1, 2, 4, 8, 16):
        got = push6(orc, v0, inputs.sext_thick(k2, length, IG2, n))
        errs.append(np.abs(got - want)[:4].max())
    ratios = [errs[i] / errs[i + 1] for i in range(len(errs) - 1)]
    assert all(3.0 < r < 20.0 for r in ratios), (errs, ratios)
    assert errs[-1] < errs[0] / 150  # 16x smaller step: 256x at second order


def test_thick_elements_need_longitudinal_arrays(orc):
    p = {k: np.zeros(4) for k in ("x", "px", "y", "py")}
    with pytest.raises(ValueError):
        orc.push(p, inputs.quad_thick(1.0, 0.5, IG2))
    p6 = dict(p, sigma=np.zeros(4), psigma=np.zeros(4))
    with pytest.raises(ValueError):
        orc.push(p6, inputs.sext_thick(1.0, 0.5, IG2, 0))


def test_linear_elements_leave_longitudinal_coordinates_alone(orc):
    w = inputs.gaussian_beam6d(100, 3)
    s0 = w["sigma"].copy()
    ps0 = w["psigma"].copy()
    orc.push(w, inputs.ring(4.2, 4.3, 8, kappa=None, k2l=3.0, sext_every=2))
    np.testing.assert_array_equal(w["sigma"], s0)
    np.testing.assert_array_equal(w["psigma"], ps0)


def test_thick_ring_one_turn_conserves_h_approx_in_each_quad(orc):
    """H_approx is an invariant of each quadrupole's flow (no s dependence
    inside the element): check it over a batch of particles."""
    b = inputs.gaussian_beam6d(2000, 11, sigma_ps=5e-3)
    v = np.stack([b[k] for k in ("x", "px", "y", "py", "sigma", "psigma")])
    h0 = h_approx(v, 0.6, 0.0, IG2)
    orc.push(b, inputs.quad_thick(0.6, 2.5, IG2))
    v1 = np.stack([b[k] for k in ("x", "px", "y", "py", "sigma", "psigma")])
    h1 = h_approx(v1, 0.6, 0.0, IG2)
    assert np.abs(h1 - h0).max() <= 1e-13 * np.abs(h0).max()
    assert math.isfinite(h1.sum())


def test_thick_sextupole_split_error_is_quadratic_in_strength(orc):
    """What the SABA2 coefficients buy (Sec. III-C, eq. Sym2): for H0 + V with
    a weak V the split's error has no term linear in the strength of V, so 10x
    the strength gives about 100x the error.  Any other symmetric
    second-order split of the same form (e.g. a and c exchanged, or leapfrog)
    errs linearly in the strength: about 10x."""
    v0 = np.array([4e-3, 1e-3, -3e-3, 5e-4, 0.1, 0.02])
    errs = []
    for k2 in (1.0, 10.0):
        want = integrate(v0, 0.5, k2=k2)
        got = push6(orc, v0, inputs.sext_thick(k2, 0.5, IG2, 2))
        errs.append(np.abs(got - want)[:4].max())
    assert 70.0 < errs[1] / errs[0] < 130.0, errs
