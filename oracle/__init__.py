"""FP64 CPU oracle of the 2D particle-in-cell space-charge step.

TEST INFRASTRUCTURE ONLY.  Only the tests, the package smoke check and the
benchmark's CPU-baseline leg may import this module.  The product path (the
HIP library and its Python binding) never imports, links or calls it, and it
shares no code with that path.

The arithmetic lives in ``scpic_oracle.c`` (plain C, FP64, no fused
multiply-add, OpenMP over particles / target nodes).  This file only builds it
with gcc and marshals numpy arrays through ctypes.

What each function follows (arXiv:2010.11540):
  push        Sec. III: transfer map per element, linear (v <- M v), the kick
              step of the split thick sextupole (Sec. III-C, potential V), the
              chromatic thick quadrupole (Sec. III-B, closed form, with the
              path-length integral for sigma) or the thick sextupole as the
              symmetric five-flow product of Sec. III-C (eq. Sym2).
  deposit     Sec. IV-A: bilinear (cloud-in-cell) charge assignment to the four
              nodes of a cell, in 2^-24 fixed-point charge units.
  potential   open-boundary Poisson solve by convolution with the free-space
              Green's function -ln r (Hockney's method, cited in Sec. I), as a
              direct sum over charged nodes; or the grounded rectangular pipe
              of Sec. IV-B (5-point Laplacian, u = 0 on the walls), written out
              as its discrete sine-eigenvector expansion.
  field       E = -grad(u) (Sec. IV-C), by centred differences on the nodes;
              or (gather="bspline") the analytic gradient of the bicubic
              surface through the 4x4 nodes around the particle's cell (the
              interpolation of Sec. IV-C read as the uniform cubic B-spline
              with the node potentials as control points).
  kick        Sec. IV: transverse kick proportional to the field at the
              particle times the distance since the previous kick, and (2.5D
              form) to the line density at the particle relative to its peak.
  line        Sec. IV: the line density lambda(sigma) as a histogram of sigma
              (the one-dimensional form of the charge assignment), recomputed
              at every space-charge step; the transverse kick scaled by
              lambda/lambda_peak and the longitudinal kick
              -gamma0 kappa phi lambda'/lambda_peak (the two printed kick
              coefficients differ by gamma0), with phi the grounded-pipe
              potential (Sec. IV-B).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from pathlib import Path

import numpy as np

_HERE = Path(__file__).resolve().parent
_SRC = _HERE / "scpic_oracle.c"
_LIB = _HERE / "liborc.so"

LIN2X2, LIN4X4, SEXT_THIN, SC, QUAD_THICK, SEXT_THICK = 1, 2, 3, 4, 5, 6
CHARGE_ONE = 1 << 24

_C_FLAGS = ["-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
            "-Wall", "-Wshadow", "-Werror"]


def build(force: bool = True) -> Path:
    """Compile the oracle with gcc into oracle/liborc.so."""
    if force or not _LIB.exists() or _LIB.stat().st_mtime < _SRC.stat().st_mtime:
        tmp = _LIB.with_suffix(".so.tmp")
        subprocess.run(["gcc", *_C_FLAGS, str(_SRC), "-o", str(tmp), "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = ctypes.CDLL(str(_LIB))
        i64, i32, dbl, vp = ctypes.c_int64, ctypes.c_int, ctypes.c_double, ctypes.c_void_p
        L.orc_num_threads.restype = i32
        L.orc_set_num_threads.argtypes = [i32]
        L.orc_set_num_threads.restype = i32
        L.orc_push.argtypes = [i64, vp, vp, vp, vp, vp, vp, vp, i32, vp, vp]
        L.orc_push.restype = i32
        L.orc_deposit.argtypes = [i64, vp, vp, vp, i32, i32, dbl, dbl, dbl, dbl, vp]
        L.orc_deposit.restype = i64
        L.orc_green.argtypes = [i32, i32, dbl, dbl]
        L.orc_green.restype = dbl
        L.orc_potential.argtypes = [vp, dbl, i32, i32, dbl, dbl, vp]
        L.orc_potential.restype = None
        L.orc_potential_pipe.argtypes = [vp, dbl, i32, i32, dbl, dbl, vp]
        L.orc_potential_pipe.restype = None
        L.orc_field.argtypes = [vp, i32, i32, dbl, dbl, vp, vp]
        L.orc_field.restype = None
        L.orc_kick.argtypes = [i64, vp, vp, vp, vp, vp, vp, i32, i32, dbl, dbl, dbl, dbl, vp, vp,
                               dbl]
        L.orc_kick.restype = None
        L.orc_space_charge.argtypes = [i64, vp, vp, vp, vp, vp, vp, i32, i32, dbl, dbl, dbl, dbl,
                                       dbl, dbl, vp, vp, i32]
        L.orc_space_charge.restype = i64
        L.orc_track.argtypes = [i64, vp, vp, vp, vp, vp, vp, vp, vp, i32, i32, dbl, dbl, dbl, dbl,
                                i32, vp, vp, i32, i32]
        L.orc_track.restype = i32
        L.orc_bspline_eval.argtypes = [i64, vp, vp, vp, i32, i32, dbl, dbl, dbl, dbl, vp, vp, vp]
        L.orc_bspline_eval.restype = None
        L.orc_kick_bspline.argtypes = [i64, vp, vp, vp, vp, vp, vp, i32, i32, dbl, dbl, dbl, dbl,
                                       vp, dbl]
        L.orc_kick_bspline.restype = None
        L.orc_space_charge_bspline.argtypes = [i64, vp, vp, vp, vp, vp, vp, i32, i32, dbl, dbl,
                                               dbl, dbl, dbl, dbl, i32]
        L.orc_space_charge_bspline.restype = i64
        L.orc_track_gather.argtypes = [i64, vp, vp, vp, vp, vp, vp, vp, vp, i32, i32, dbl, dbl, dbl,
                                       dbl, i32, vp, vp, i32, i32, i32]
        L.orc_track_gather.restype = i32
        L.orc_deposit_line.argtypes = [i64, vp, vp, vp, vp, i32, i32, dbl, dbl, dbl, dbl, i32, dbl,
                                       dbl, vp, vp]
        L.orc_deposit_line.restype = i64
        L.orc_line_table.argtypes = [vp, i32, dbl, vp, vp]
        L.orc_line_table.restype = None
        L.orc_space_charge_line.argtypes = [i64, vp, vp, vp, vp, vp, vp, vp, i32, i32, dbl, dbl, dbl,
                                            dbl, i32, dbl, dbl, dbl, dbl, dbl, vp, vp, vp]
        L.orc_space_charge_line.restype = i64
        L.orc_track_line.argtypes = [i64, vp, vp, vp, vp, vp, vp, vp, i32, i32, dbl, dbl, dbl, dbl,
                                     i32, dbl, dbl, dbl, i32, vp, vp, i32]
        L.orc_track_line.restype = i32
        _lib = L
    return _lib


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a


def _ptr(a):
    return None if a is None else a.ctypes.data


def _grid_args(grid):
    return (int(grid["nx"]), int(grid["ny"]), float(grid["x_min"]), float(grid["y_min"]),
            float(grid["dx"]), float(grid["dy"]))


def _elements(elements):
    kind = np.ascontiguousarray(elements["kind"], dtype=np.int32)
    par = np.ascontiguousarray(elements["p"], dtype=np.float64).reshape(-1, 16)
    return kind, par


def num_threads() -> int:
    return lib().orc_num_threads()


def set_num_threads(n: int) -> int:
    """OpenMP threads of later oracle calls (timing only); returns the count in effect."""
    return lib().orc_set_num_threads(int(n))


def _longitudinal(parts):
    s, ps = parts.get("sigma"), parts.get("psigma")
    for a in (s, ps):
        if a is not None and (a.dtype != np.float64 or not a.flags.c_contiguous):
            raise TypeError("sigma and psigma must be contiguous float64 arrays")
    return _ptr(s), _ptr(ps)


def push(parts: dict, elements) -> None:
    """In place: push particles through the non-space-charge elements.  Thick
    elements need parts['sigma'] and parts['psigma']."""
    kind, par = _elements(elements)
    n = parts["x"].shape[0]
    rc = lib().orc_push(n, _ptr(parts["x"]), _ptr(parts["px"]), _ptr(parts["y"]),
                        _ptr(parts["py"]), *_longitudinal(parts), _ptr(parts.get("lost")),
                        len(kind), _ptr(kind), _ptr(par))
    if rc != 0:
        raise ValueError("thick elements need sigma and psigma, and n >= 1 sextupole steps")


def deposit(parts: dict, grid) -> tuple[np.ndarray, int]:
    """Charge grid q (int64, nx*ny, 2^24 units per particle) and number deposited.
    Marks out-of-domain particles lost when parts has a 'lost' array."""
    nx, ny = int(grid["nx"]), int(grid["ny"])
    q = np.zeros(nx * ny, dtype=np.int64)
    n = parts["x"].shape[0]
    n_in = lib().orc_deposit(n, _ptr(parts["x"]), _ptr(parts["y"]), _ptr(parts.get("lost")),
                             *_grid_args(grid), _ptr(q))
    if n_in < 0:
        raise MemoryError("oracle deposit: allocation failed")
    return q, int(n_in)


def green(di: int, dj: int, dx: float, dy: float) -> float:
    return lib().orc_green(di, dj, dx, dy)


def potential(q: np.ndarray, scale: float, grid, solver: str = "open") -> np.ndarray:
    """phi on nodes -1..nx, -1..ny as an (nx+2, ny+2) array: the open-boundary
    convolution (solver="open") or the grounded pipe with walls through node 0
    and node n of each axis (solver="pipe")."""
    nx, ny = int(grid["nx"]), int(grid["ny"])
    q = np.ascontiguousarray(q, dtype=np.int64)
    phi = np.zeros((nx + 2) * (ny + 2), dtype=np.float64)
    fn = {"open": lib().orc_potential, "pipe": lib().orc_potential_pipe}[solver]
    fn(_ptr(q), float(scale), nx, ny, float(grid["dx"]), float(grid["dy"]), _ptr(phi))
    return phi.reshape(nx + 2, ny + 2)


def field(phi: np.ndarray, grid) -> tuple[np.ndarray, np.ndarray]:
    """(ex, ey), each nx*ny row-major."""
    nx, ny = int(grid["nx"]), int(grid["ny"])
    phi = _f64(phi)
    ex = np.zeros(nx * ny)
    ey = np.zeros(nx * ny)
    lib().orc_field(_ptr(phi), nx, ny, float(grid["dx"]), float(grid["dy"]), _ptr(ex), _ptr(ey))
    return ex, ey


def solve(q: np.ndarray, scale: float, grid, solver: str = "open") -> tuple[np.ndarray, np.ndarray]:
    """Field on the nodes from a charge grid: potential then centred differences."""
    return field(potential(q, scale, grid, solver), grid)


def _weights(parts):
    w = parts.get("w")
    if w is None:
        return None
    if w.dtype != np.float32 or not w.flags.c_contiguous:
        raise TypeError("w must be a contiguous float32 array")
    return w


def kick(parts: dict, grid, ex: np.ndarray, ey: np.ndarray, kappa: float) -> None:
    """In place: gather the node field with the deposit weights,
    p += kappa * w_p * E (w_p = parts['w'] when present, else 1)."""
    n = parts["x"].shape[0]
    ex = _f64(ex)
    ey = _f64(ey)
    lib().orc_kick(n, _ptr(parts["x"]), _ptr(parts["px"]), _ptr(parts["y"]), _ptr(parts["py"]),
                   _ptr(parts.get("lost")), _ptr(_weights(parts)), *_grid_args(grid), _ptr(ex),
                   _ptr(ey), float(kappa))


def bspline_eval(x: np.ndarray, y: np.ndarray, phi: np.ndarray, grid):
    """(u, ex, ey) of the B-spline surface of the node potential phi (as
    potential() returns it) at the points; NaN outside the domain."""
    x, y = _f64(x), _f64(y)
    phi = _f64(phi).ravel()
    n = x.shape[0]
    u, ex, ey = np.zeros(n), np.zeros(n), np.zeros(n)
    lib().orc_bspline_eval(n, _ptr(x), _ptr(y), _ptr(phi), *_grid_args(grid), _ptr(u), _ptr(ex),
                           _ptr(ey))
    return u, ex, ey


def space_charge(parts: dict, grid, scale: float, kappa: float, solver: str = "open",
                 gather: str = "cic"):
    """One full space-charge step in place; returns (ex, ey, n_in) (the node
    field; with gather="bspline" the kick takes the B-spline gradient instead
    and (None, None, n_in) is returned)."""
    if gather == "bspline":
        n = parts["x"].shape[0]
        n_in = lib().orc_space_charge_bspline(n, _ptr(parts["x"]), _ptr(parts["px"]),
                                              _ptr(parts["y"]), _ptr(parts["py"]),
                                              _ptr(parts.get("lost")), _ptr(_weights(parts)),
                                              *_grid_args(grid), float(scale), float(kappa),
                                              _pipe(solver))
        return None, None, int(n_in)
    nx, ny = int(grid["nx"]), int(grid["ny"])
    ex = np.zeros(nx * ny)
    ey = np.zeros(nx * ny)
    n = parts["x"].shape[0]
    n_in = lib().orc_space_charge(n, _ptr(parts["x"]), _ptr(parts["px"]), _ptr(parts["y"]),
                                  _ptr(parts["py"]), _ptr(parts.get("lost")),
                                  _ptr(_weights(parts)), *_grid_args(grid), float(scale),
                                  float(kappa), _ptr(ex), _ptr(ey), _pipe(solver))
    return ex, ey, int(n_in)


def _pipe(solver: str) -> int:
    return {"open": 0, "pipe": 1}[solver]


def track(parts: dict, grid, elements, n_turns: int, solver: str = "open",
          gather: str = "cic") -> None:
    """In place: n_turns through the one-turn element sequence."""
    kind, par = _elements(elements)
    n = parts["x"].shape[0]
    rc = lib().orc_track_gather(n, _ptr(parts["x"]), _ptr(parts["px"]), _ptr(parts["y"]),
                                _ptr(parts["py"]), *_longitudinal(parts), _ptr(parts.get("lost")),
                                _ptr(_weights(parts)), *_grid_args(grid), len(kind), _ptr(kind),
                                _ptr(par), int(n_turns), _pipe(solver),
                                {"cic": 0, "bspline": 1}[gather])
    if rc != 0:
        raise ValueError("thick elements need sigma and psigma, and n >= 1 sextupole steps")


def _line_args(line):
    return int(line["nz"]), float(line["z_min"]), float(line["dz"])


def deposit_line(parts: dict, grid, line) -> tuple[np.ndarray, np.ndarray, int]:
    """Transverse charge q (nx*ny) and line histogram h (nz, 4096 units per
    particle) of the particles inside both domains; the others are marked lost."""
    nx, ny = int(grid["nx"]), int(grid["ny"])
    q = np.zeros(nx * ny, dtype=np.int64)
    h = np.zeros(int(line["nz"]), dtype=np.int64)
    n = parts["x"].shape[0]
    n_in = lib().orc_deposit_line(n, _ptr(parts["x"]), _ptr(parts["y"]), _ptr(_f64(parts["sigma"])),
                                  _ptr(parts.get("lost")), *_grid_args(grid), *_line_args(line),
                                  _ptr(q), _ptr(h))
    return q, h, int(n_in)


def line_table(h: np.ndarray, line) -> tuple[np.ndarray, np.ndarray]:
    """(lambda/lambda_peak, lambda'/lambda_peak) at the line's nodes."""
    h = np.ascontiguousarray(h, dtype=np.int64)
    nz = int(line["nz"])
    lw, ld = np.zeros(nz), np.zeros(nz)
    lib().orc_line_table(_ptr(h), nz, float(line["dz"]), _ptr(lw), _ptr(ld))
    return lw, ld


def space_charge_line(parts: dict, grid, line, scale: float, kappa: float):
    """One long-bunch space-charge step in place (grounded pipe); returns
    (lw, ld, phi, n_in) with phi as potential(..., solver="pipe")."""
    nx, ny = int(grid["nx"]), int(grid["ny"])
    nz = int(line["nz"])
    lw, ld = np.zeros(nz), np.zeros(nz)
    phi = np.zeros((nx + 2) * (ny + 2))
    n = parts["x"].shape[0]
    sp, psp = _longitudinal(parts)
    if sp is None or psp is None:
        raise ValueError("the line-density step needs sigma and psigma")
    n_in = lib().orc_space_charge_line(n, _ptr(parts["x"]), _ptr(parts["px"]), _ptr(parts["y"]),
                                       _ptr(parts["py"]), sp, psp, _ptr(parts.get("lost")),
                                       *_grid_args(grid), *_line_args(line), float(line["gamma0"]),
                                       float(scale), float(kappa), _ptr(lw), _ptr(ld), _ptr(phi))
    if n_in < 0:
        raise MemoryError("oracle line step: allocation failed")
    return lw, ld, phi.reshape(nx + 2, ny + 2), int(n_in)


def track_line(parts: dict, grid, line, elements, n_turns: int) -> None:
    """In place: n_turns with the long-bunch space-charge step (grounded pipe)
    at every SC element."""
    kind, par = _elements(elements)
    n = parts["x"].shape[0]
    sp, psp = _longitudinal(parts)
    if sp is None or psp is None:
        raise ValueError("the line-density step needs sigma and psigma")
    rc = lib().orc_track_line(n, _ptr(parts["x"]), _ptr(parts["px"]), _ptr(parts["y"]),
                              _ptr(parts["py"]), sp, psp, _ptr(parts.get("lost")),
                              *_grid_args(grid), *_line_args(line), float(line["gamma0"]),
                              len(kind), _ptr(kind), _ptr(par), int(n_turns))
    if rc != 0:
        raise ValueError("bad sextupole steps or out of memory")
