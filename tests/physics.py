"""Test-side diagnostics and closed forms (no part of the method's arithmetic).

Closed forms used as pins, in the oracle's normalisation (lap phi = -2 pi rho,
total charge Q, E = -grad phi):
  * round Gaussian, rms sigma:    E_r(r) = Q (1 - exp(-r^2 / 2 sigma^2)) / r
  * uniform ellipse, semi-axes a, b, inside:
                                  E_x = 2 Q x / (a (a + b)),  E_y = 2 Q y / (b (a + b))
  * point charge:                 E_r(r) = Q / r
"""
from __future__ import annotations

import math

import numpy as np


def rms_emittance(u: np.ndarray, pu: np.ndarray, alive: np.ndarray | None = None) -> float:
    if alive is not None:
        u, pu = u[alive], pu[alive]
    du = u - u.mean()
    dp = pu - pu.mean()
    a = np.mean(du * du)
    b = np.mean(dp * dp)
    c = np.mean(du * dp)
    return math.sqrt(a * b - c * c)


def gaussian_er(r, sigma, q=1.0):
    r = np.asarray(r, dtype=np.float64)
    out = np.empty_like(r)
    small = r < 1e-12
    out[small] = 0.0
    rs = r[~small]
    out[~small] = q * (-np.expm1(-rs * rs / (2 * sigma * sigma))) / rs
    return out


def ellipse_field(x, y, a, b, q=1.0):
    return 2 * q * x / (a * (a + b)), 2 * q * y / (b * (a + b))


def tune_from_turns(xs: np.ndarray, pxs: np.ndarray, beta: float = 1.0) -> float:
    """Fractional tune from turn-by-turn (x, px) at a symmetry point with
    alpha = 0: mean phase advance per turn of the normalised phase-space vector
    (x/sqrt(beta), sqrt(beta) px), turning clockwise."""
    ang = np.arctan2(-np.asarray(pxs) * math.sqrt(beta), np.asarray(xs) / math.sqrt(beta))
    d = np.mod(np.diff(ang), 2 * math.pi)
    return float(np.mean(d) / (2 * math.pi))


def thin_lens_ring_tune(mu: float, k: float, n_seg: int, beta: float = 1.0) -> float:
    """Fractional tune of n_seg x [rotation(mu); thin lens p += k x] from the
    one-turn matrix trace (k > 0 defocusing)."""
    c, s = math.cos(mu), math.sin(mu)
    r = np.array([[c, beta * s], [-s / beta, c]])
    lens = np.array([[1.0, 0.0], [k, 1.0]])
    m = np.eye(2)
    for _ in range(n_seg):
        m = lens @ r @ m
    cos_mu = 0.5 * np.trace(m)
    frac = math.acos(max(-1.0, min(1.0, cos_mu))) / (2 * math.pi)
    return frac


def laslett_tune_shift(n_ppb, harmonic, r_p, beta0, gamma0, eps_1sigma, bunch_factor):
    """Incoherent tune spread estimate of a Gaussian bunch (Sec. V)."""
    return -n_ppb * harmonic * r_p / (4 * math.pi * beta0 ** 2 * gamma0 ** 3 * eps_1sigma
                                      * bunch_factor)


def record_figures(name: str, figures: dict) -> None:
    """Keep a test's printed figures: merged into gpurun_out/test_figures.json
    at the repository root (one entry per name, overwritten by a rerun)."""
    import json
    from pathlib import Path

    out = Path(__file__).resolve().parent.parent / "gpurun_out" / "test_figures.json"
    out.parent.mkdir(exist_ok=True)
    try:
        data = json.loads(out.read_text())
    except (OSError, ValueError):
        data = {}
    data[name] = figures
    out.write_text(json.dumps(data, indent=1, sort_keys=True))
