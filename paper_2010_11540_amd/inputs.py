"""Seeded synthetic inputs: beams, grids and ring lattices.

This module only *describes* workloads.  It draws particle coordinates from
seeded numpy generators and writes lattice element tables; it performs none of
the space-charge step's arithmetic (no push, deposit, solve or kick), so both
the HIP path and the CPU oracle can take their inputs from it without sharing
any of the method.

Workload recipes (stand-ins for the paper's J-PARC Main Ring runs, whose
lattice and measured beam are not public):
  * round Gaussian beam, sigma_x = sigma_y = 1 mm, sigma_x' = sigma_y' = 1 mrad
    (beta = 1 m, alpha = 0 at every space-charge location, matched);
  * grid of N x N nodes spanning +-6 sigma;
  * ring of identical segments, each one phase-advance rotation per plane
    (tunes Q_x, Q_y split evenly over the segments), optional thin sextupoles,
    one space-charge kick per segment;
  * kick coefficient set from a target incoherent tune shift with the
    smooth-focusing Laslett relation for a Gaussian beam (Sec. V, tune-spread
    estimate): dnu = -K C / (8 pi eps_rms).
"""
from __future__ import annotations

import math

import numpy as np

# element kinds (same numbering as the C ABI's scpic_element_kind)
LIN2X2, LIN4X4, SEXT_THIN, SC, QUAD_THICK, SEXT_THICK = 1, 2, 3, 4, 5, 6

ELEMENT_DTYPE = np.dtype([("kind", "<i4"), ("pad", "<i4"), ("p", "<f8", (16,))], align=True)
assert ELEMENT_DTYPE.itemsize == 136

SEED_BASE = 2010_11540

# proton rest energy [GeV] and classical proton radius [m] (CODATA 2018)
PROTON_MASS_GEV = 0.93827208816
PROTON_RADIUS_M = 1.53469857e-18


# --------------------------------------------------------------------------
# grids
# --------------------------------------------------------------------------

def make_grid(nx: int, ny: int | None = None, half_x: float = 6e-3, half_y: float | None = None,
              center_x: float = 0.0, center_y: float = 0.0) -> dict:
    """nx x ny nodes spanning [center - half, center + half] in each plane."""
    ny = nx if ny is None else ny
    half_y = half_x if half_y is None else half_y
    return {
        "nx": int(nx), "ny": int(ny),
        "x_min": center_x - half_x, "y_min": center_y - half_y,
        "dx": 2.0 * half_x / (nx - 1), "dy": 2.0 * half_y / (ny - 1),
    }


# --------------------------------------------------------------------------
# beams
# --------------------------------------------------------------------------

def gaussian_beam(n: int, seed: int, sigma_x=1e-3, sigma_px=1e-3, sigma_y=1e-3, sigma_py=1e-3,
                  lost: bool = True) -> dict:
    rng = np.random.Generator(np.random.PCG64(seed))
    z = rng.standard_normal((4, n))
    parts = {
        "x": np.ascontiguousarray(z[0] * sigma_x),
        "px": np.ascontiguousarray(z[1] * sigma_px),
        "y": np.ascontiguousarray(z[2] * sigma_y),
        "py": np.ascontiguousarray(z[3] * sigma_py),
    }
    if lost:
        parts["lost"] = np.zeros(n, dtype=np.uint8)
    return parts


def gaussian_beam6d(n: int, seed: int, sigma_x=1e-3, sigma_px=1e-3, sigma_y=1e-3, sigma_py=1e-3,
                    sigma_z=1.0, sigma_ps=1e-3, lost: bool = True) -> dict:
    """Gaussian in all six canonical coordinates (x, px, y, py, sigma, p_sigma),
    uncorrelated: the transverse part of a long bunch with a momentum spread."""
    rng = np.random.Generator(np.random.PCG64(seed))
    z = rng.standard_normal((6, n))
    parts = {
        "x": np.ascontiguousarray(z[0] * sigma_x),
        "px": np.ascontiguousarray(z[1] * sigma_px),
        "y": np.ascontiguousarray(z[2] * sigma_y),
        "py": np.ascontiguousarray(z[3] * sigma_py),
        "sigma": np.ascontiguousarray(z[4] * sigma_z),
        "psigma": np.ascontiguousarray(z[5] * sigma_ps),
    }
    if lost:
        parts["lost"] = np.zeros(n, dtype=np.uint8)
    return parts


def kv_beam(n: int, seed: int, a=4e-3, b=2e-3, beta_x=1.0, beta_y=1.0, lost: bool = True) -> dict:
    """Kapchinskij-Vladimirskij beam: uniform on the surface of a 4D ellipsoid,
    so its x-y projection is a uniform ellipse with semi-axes a, b."""
    rng = np.random.Generator(np.random.PCG64(seed))
    g = rng.standard_normal((4, n))
    u = g / np.linalg.norm(g, axis=0)
    parts = {
        "x": np.ascontiguousarray(a * u[0]),
        "px": np.ascontiguousarray(a / beta_x * u[1]),
        "y": np.ascontiguousarray(b * u[2]),
        "py": np.ascontiguousarray(b / beta_y * u[3]),
    }
    if lost:
        parts["lost"] = np.zeros(n, dtype=np.uint8)
    return parts


def line_density_weights(z: np.ndarray, z_half: float, bins: int = 128) -> np.ndarray:
    """Static 2.5D kick weights: the line density lambda(z) of the bunch as a
    histogram of z over [-z_half, z_half] (the paper uses 128 bins, Sec. IV),
    divided by its peak, read at each particle's bin."""
    counts, edges = np.histogram(z, bins=bins, range=(-z_half, z_half))
    k = np.clip(((z + z_half) / (2 * z_half) * bins).astype(np.int64), 0, bins - 1)
    return np.ascontiguousarray(counts[k] / counts.max(), dtype=np.float32)


def long_bunch_kv(n: int, seed: int, a=4e-3, b=2e-3, beta=1.0, sigma_z=0.25, z_half=0.5) -> dict:
    """KV transverse beam with a Gaussian longitudinal profile (rms sigma_z in
    bucket units, truncated to +-z_half) turned into per-particle kick weights."""
    parts = kv_beam(n, seed, a, b, beta, beta)
    rng = np.random.Generator(np.random.PCG64(seed + 7919))
    z = rng.standard_normal(2 * n + 1000) * sigma_z
    z = z[np.abs(z) < z_half][:n]
    while z.shape[0] < n:  # practically never: the cut keeps ~95% of draws
        more = rng.standard_normal(n) * sigma_z
        z = np.concatenate([z, more[np.abs(more) < z_half]])[:n]
    parts["w"] = line_density_weights(z, z_half)
    parts["z"] = np.ascontiguousarray(z)
    return parts


def uniform_in_box(n: int, seed: int, grid: dict, margin: float = 0.0) -> dict:
    """Positions uniform over the grid's domain (shrunk by margin cells)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lx = (grid["nx"] - 1) * grid["dx"]
    ly = (grid["ny"] - 1) * grid["dy"]
    x = grid["x_min"] + margin * grid["dx"] + rng.random(n) * (lx - 2 * margin * grid["dx"])
    y = grid["y_min"] + margin * grid["dy"] + rng.random(n) * (ly - 2 * margin * grid["dy"])
    return {"x": x, "px": rng.standard_normal(n) * 1e-3, "y": y,
            "py": rng.standard_normal(n) * 1e-3, "lost": np.zeros(n, dtype=np.uint8)}


# --------------------------------------------------------------------------
# lattices
# --------------------------------------------------------------------------

def elements(n: int) -> np.ndarray:
    return np.zeros(n, dtype=ELEMENT_DTYPE)


def rotation(mu: float, beta: float = 1.0, alpha: float = 0.0) -> np.ndarray:
    """Courant-Snyder phase-advance matrix of one plane (det = 1)."""
    c, s = math.cos(mu), math.sin(mu)
    gamma = (1.0 + alpha * alpha) / beta
    return np.array([[c + alpha * s, beta * s], [-gamma * s, c - alpha * s]])


def lin2x2(mx: np.ndarray, my: np.ndarray) -> np.ndarray:
    e = elements(1)
    e["kind"] = LIN2X2
    e["p"][0, 0:4] = np.asarray(mx, dtype=np.float64).reshape(4)
    e["p"][0, 4:8] = np.asarray(my, dtype=np.float64).reshape(4)
    return e


def lin4x4(m: np.ndarray) -> np.ndarray:
    e = elements(1)
    e["kind"] = LIN4X4
    e["p"][0, :] = np.asarray(m, dtype=np.float64).reshape(16)
    return e


def sext_thin(k2l: float) -> np.ndarray:
    e = elements(1)
    e["kind"] = SEXT_THIN
    e["p"][0, 0] = k2l
    return e


def quad_thick(k1: float, length: float, inv_gamma2: float) -> np.ndarray:
    """Thick quadrupole with chromatic focusing (Sec. III-B); k1 > 0 focuses x."""
    e = elements(1)
    e["kind"] = QUAD_THICK
    e["p"][0, :3] = (k1, length, inv_gamma2)
    return e


def sext_thick(k2: float, length: float, inv_gamma2: float, steps: int = 1) -> np.ndarray:
    """Thick sextupole by the symmetric split of Sec. III-C, applied `steps`
    times over length/steps; k2 = 0 is the exact drift of H0."""
    e = elements(1)
    e["kind"] = SEXT_THICK
    e["p"][0, :4] = (k2, length, inv_gamma2, float(steps))
    return e


def drift(length: float, inv_gamma2: float) -> np.ndarray:
    return sext_thick(0.0, length, inv_gamma2, 1)


def sc_kick(kappa: float) -> np.ndarray:
    e = elements(1)
    e["kind"] = SC
    e["p"][0, 0] = kappa
    return e


def block_diag4(mx: np.ndarray, my: np.ndarray) -> np.ndarray:
    m = np.zeros((4, 4))
    m[0:2, 0:2] = mx
    m[2:4, 2:4] = my
    return m


def random_symplectic4(seed: int, scale: float = 0.3) -> np.ndarray:
    """A coupled 4x4 symplectic matrix exp(J S), S random symmetric."""
    from scipy.linalg import expm
    rng = np.random.Generator(np.random.PCG64(seed))
    a = rng.standard_normal((4, 4)) * scale
    s = a + a.T
    j = np.array([[0, 1, 0, 0], [-1, 0, 0, 0], [0, 0, 0, 1], [0, 0, -1, 0]], dtype=np.float64)
    return expm(j @ s)


def kappa_for_tune_shift(dnu: float, eps_rms: float, n_kicks: int) -> float:
    """Kick coefficient per space-charge location giving the incoherent
    small-amplitude tune shift dnu (< 0) of a round Gaussian beam with rms
    emittance eps_rms, in the smooth approximation: K C = 8 pi eps |dnu|."""
    return 8.0 * math.pi * eps_rms * abs(dnu) / n_kicks


def ring(qx: float, qy: float, n_seg: int, kappa: float, beta: float = 1.0,
         four_by_four: bool = False, k2l: float = 0.0, sext_every: int = 0,
         coupled: np.ndarray | None = None) -> np.ndarray:
    """One turn of n_seg identical segments: [map; (thin sextupole); SC kick].

    The map advances the phase by 2 pi q / n_seg per plane (LIN2X2, or the same
    as a block-diagonal LIN4X4).  With sext_every > 0, a thin sextupole of
    strength k2l follows the map of every sext_every-th segment (1-based).
    coupled, when given, replaces the map of the first segment (LIN4X4)."""
    mx = rotation(2.0 * math.pi * qx / n_seg, beta)
    my = rotation(2.0 * math.pi * qy / n_seg, beta)
    parts = []
    for k in range(1, n_seg + 1):
        if coupled is not None and k == 1:
            parts.append(lin4x4(coupled))
        elif four_by_four:
            parts.append(lin4x4(block_diag4(mx, my)))
        else:
            parts.append(lin2x2(mx, my))
        if sext_every and k % sext_every == 0:
            parts.append(sext_thin(k2l))
        if kappa is not None:
            parts.append(sc_kick(kappa))
    return np.concatenate(parts)


def make_line(half: float, nz: int = 128, gamma0: float | None = None) -> dict:
    """Line-density grid of nz nodes spanning [-half, half] in sigma (the
    paper's 128-bin line density, Sec. IV), with the reference gamma0 of the
    longitudinal kick."""
    return {"nz": int(nz), "z_min": -half, "dz": 2.0 * half / (nz - 1),
            "gamma0": GAMMA0_3GEV if gamma0 is None else float(gamma0)}


# 3 GeV kinetic energy protons (the Main Ring's injection energy)
GAMMA0_3GEV = 1.0 + 3.0 / PROTON_MASS_GEV


def fodo_thick(n_cell: int, q: float, kappa: float | None, cell_length: float = 4.0,
               quad_length: float = 0.5, sext_length: float = 0.2, k2f: float = 20.0,
               k2d: float = -30.0, gamma0: float = GAMMA0_3GEV, sext_steps: int = 1) -> np.ndarray:
    """One turn of n_cell thick FODO cells, each
         [QF/2, D, SF, D, QD, D, SD, D, QF/2, SC kick]
    (the kick sits at the middle of QF, where alpha = 0).  The quadrupole
    gradient is set from the thin-lens FODO relation for a phase advance of
    2 pi q / n_cell per cell, f = L_cell / (4 sin(mu/2)), k1 = 1 / (f L_quad);
    the thick magnets make the actual advance slightly different."""
    ig2 = 1.0 / (gamma0 * gamma0)
    mu = 2.0 * math.pi * q / n_cell
    k1 = 4.0 * math.sin(0.5 * mu) / (cell_length * quad_length)
    d = 0.25 * (cell_length - 2.0 * quad_length - 2.0 * sext_length)
    cell = [quad_thick(k1, 0.5 * quad_length, ig2), drift(d, ig2),
            sext_thick(k2f, sext_length, ig2, sext_steps), drift(d, ig2),
            quad_thick(-k1, quad_length, ig2), drift(d, ig2),
            sext_thick(k2d, sext_length, ig2, sext_steps), drift(d, ig2),
            quad_thick(k1, 0.5 * quad_length, ig2)]
    if kappa is not None:
        cell.append(sc_kick(kappa))
    return np.concatenate(cell * n_cell)


def fodo_beta(n_cell: int, q: float, cell_length: float = 4.0) -> tuple[float, float]:
    """Thin-lens FODO beta at the focusing and defocusing quadrupole centres."""
    mu = 2.0 * math.pi * q / n_cell
    s = math.sin(0.5 * mu)
    return (cell_length * (1 + s) / math.sin(mu), cell_length * (1 - s) / math.sin(mu))


# --------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------

def workload(name: str, n: int | None = None, seed: int | None = None) -> dict:
    """Particles, grid and one-turn lattice of a named workload.

    small      1e4 Gaussian, 64^2 grid over +-6 sigma, 16 segments (2x2 maps,
               Q = 4.2/4.3), one SC kick per segment, dnu = -0.2; 10 turns.
    production 1e6 Gaussian, 128^2 grid, 100 block-diagonal 4x4 maps plus 10
               thin sextupoles (k2L = 5 m^-2) and 100 SC kicks per turn,
               dnu = -0.2; 100 turns.
    large      1e7 particles, KV 2:1 (a = 4 mm, b = 2 mm) with Gaussian z
               (sigma = 0.25 bucket, cut at +-0.5) as 128-bin line-density
               kick weights, 256^2 grid over +-12 x +-6 mm (+-6 rms), 200
               segments without sextupoles, kappa for dnu_y = -0.2 at the
               bunch peak (K C = 2 pi (eps_y + sqrt(eps_x eps_y)) 0.2, edge
               emittances); 1000 turns.
    """
    eps = 1e-6  # rms emittance (1 mm x 1 mrad)
    if name == "small":
        n = 10_000 if n is None else n
        seed = SEED_BASE + 1 if seed is None else seed
        grid = make_grid(64)
        lat = ring(4.2, 4.3, 16, kappa_for_tune_shift(-0.2, eps, 16))
        turns = 10
    elif name == "production":
        n = 1_000_000 if n is None else n
        seed = SEED_BASE + 2 if seed is None else seed
        grid = make_grid(128)
        lat = ring(4.2, 4.3, 100, kappa_for_tune_shift(-0.2, eps, 100), four_by_four=True,
                   k2l=5.0, sext_every=10)
        turns = 100
    elif name == "large":
        n = 10_000_000 if n is None else n
        seed = SEED_BASE + 5 if seed is None else seed
        grid = make_grid(256, 256, 12e-3, 6e-3)
        a, b = 4e-3, 2e-3
        eps_x, eps_y = a * a, b * b  # edge emittances at beta = 1 m
        kc = 2 * math.pi * (eps_y + math.sqrt(eps_x * eps_y)) * 0.2
        lat = ring(4.2, 4.3, 200, kc / 200)
        return {"name": name, "parts": long_bunch_kv(n, seed, a, b), "grid": grid, "lattice": lat,
                "turns": 1000, "n": n, "seed": seed}
    elif name in ("line", "line_small"):
        # the thick rings with the long-bunch line density: 128 nodes over
        # +-6 sigma_z (sigma_z = 1 m), grounded-pipe solver
        w = workload("thick" if name == "line" else "thick_small", n, seed)
        w.update(name=name, line=make_line(6.0, 128), solver="pipe")
        return w
    elif name in ("thick", "thick_small"):
        # 6D beam through thick chromatic quadrupoles and SABA2 thick
        # sextupoles: 1 mm rms at the kick in both planes, p_sigma rms 1e-3
        big = name == "thick"
        n = (1_000_000 if big else 10_000) if n is None else n
        seed = SEED_BASE + (6 if big else 7) if seed is None else seed
        grid = make_grid(128 if big else 64)
        n_cell = 100 if big else 16
        bx, by = fodo_beta(n_cell, 4.2)
        eps_x = 1e-6 / bx
        lat = fodo_thick(n_cell, 4.2, kappa_for_tune_shift(-0.2, eps_x, n_cell))
        parts = gaussian_beam6d(n, seed, 1e-3, 1e-3 / bx, 1e-3 * math.sqrt(by / bx),
                                1e-3 / math.sqrt(bx * by))
        return {"name": name, "parts": parts, "grid": grid, "lattice": lat,
                "turns": 10 if big else 10, "n": n, "seed": seed}
    else:
        raise ValueError(f"unknown workload {name!r}")
    return {"name": name, "parts": gaussian_beam(n, seed), "grid": grid, "lattice": lat,
            "turns": turns, "n": n, "seed": seed}


def concat_parts(beams: list[dict]) -> tuple[dict, np.ndarray]:
    """Concatenate per-beam particle dicts (same keys) and return the CSR
    offsets of the beams."""
    keys = beams[0].keys()
    parts = {k: np.ascontiguousarray(np.concatenate([b[k] for b in beams])) for k in keys}
    offsets = np.zeros(len(beams) + 1, dtype=np.int64)
    offsets[1:] = np.cumsum([b["x"].shape[0] for b in beams])
    return parts, offsets


def batch_workload(n_inst: int = 64, seed: int | None = None, n_min: float = 1e4,
                   n_max: float = 5e5, turns: int = 200, tune_lo: float = 4.05,
                   tune_hi: float = 4.45, dnu: float = -0.2) -> dict:
    """A tune scan as one batch of independent beams (the paper's Sec. V scans
    tunes beam by beam).

    Beam k: N_k = round(10^U(log10 n_min, log10 n_max)) Gaussian particles
    (the same distribution as the other workloads, its own seed), on a 64^2
    grid over +-6 sigma when N_k < 1e5, else 128^2; its ring is the small
    workload's (16 segments of 2x2 maps, one SC kick each, kappa for the
    tune shift dnu, -0.2 by default) at the tunes (Q_x, Q_y) of point k of an s x s lattice over
    [tune_lo, tune_hi]^2 (s = ceil(sqrt(n_inst))).  Beams near the integer lose
    particles, which exercises the lost flags and uneven beam sizes."""
    seed = SEED_BASE + 4 if seed is None else seed
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.uniform(math.log10(n_min), math.log10(n_max), size=n_inst)
    sizes = np.rint(10.0 ** u).astype(np.int64)
    side = int(math.ceil(math.sqrt(n_inst)))
    q = np.linspace(tune_lo, tune_hi, side)
    eps = 1e-6
    kappa = kappa_for_tune_shift(dnu, eps, 16)
    beams, grids, lattices, tunes = [], [], [], []
    for k in range(n_inst):
        qx, qy = q[k % side], q[(k // side) % side]
        beams.append(gaussian_beam(int(sizes[k]), seed * 1000 + k))
        grids.append(make_grid(64 if sizes[k] < 100_000 else 128))
        lattices.append(ring(qx, qy, 16, kappa))
        tunes.append((qx, qy))
    parts, offsets = concat_parts(beams)
    return {"name": "batch", "parts": parts, "offsets": offsets, "grids": grids,
            "lattices": lattices, "tunes": tunes, "sizes": sizes, "turns": turns,
            "n": int(offsets[-1]), "seed": seed}


def copy_parts(parts: dict) -> dict:
    return {k: v.copy() for k, v in parts.items()}
