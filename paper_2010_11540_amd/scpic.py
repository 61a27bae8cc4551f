"""ctypes binding of libscpic (include/scpic.h) over PyTorch device tensors.

Argument marshalling only: every step of the space-charge loop runs in the HIP
kernels of libscpic.so.  Importing this module loads the library; if it has
not been built, or no GPU is present when a context is created, the call fails
loudly -- there is no CPU fallback.

Particles are a dict of contiguous 1-D CUDA tensors: x, px, y, py (float64)
and optionally lost (uint8).  Lattices are numpy arrays of
inputs.ELEMENT_DTYPE (the C struct scpic_element).
"""
from __future__ import annotations

import ctypes
from pathlib import Path

import numpy as np
import torch

from .inputs import ELEMENT_DTYPE

_LIB_PATH = Path(__file__).resolve().parent / "libscpic.so"

OK, EINVAL, ENOMEM, EHIP, EUNSUPPORTED = 0, -1, -2, -3, -4
FP64, MIXED = 0, 1
OPT_USE_GRAPH, OPT_PASS_BLOCKS, OPT_PASS_THREADS, OPT_SOLVER, OPT_GATHER = 1, 2, 3, 4, 5
GATHER_CIC, GATHER_BSPLINE = 0, 1
SOLVER_OPEN, SOLVER_PIPE = 0, 1

# every function the header declares, for load checks
EXPORTS = ("scpic_version", "scpic_last_error", "scpic_create", "scpic_destroy",
           "scpic_set_stream", "scpic_push", "scpic_deposit", "scpic_solve", "scpic_kick",
           "scpic_track", "scpic_set_option", "scpic_pass", "scpic_reduce_solve",
           "scpic_get_field", "scpic_batch_create", "scpic_batch_destroy",
           "scpic_batch_set_stream", "scpic_track_batched", "scpic_batch_autotune",
           "scpic_batch_get_field", "scpic_set_line_density", "scpic_get_line_state",
           "scpic_get_potential", "scpic_diagnose", "scpic_deposit_static")

# bytes of the static device scratch behind scpic_deposit_static (per device)
STATIC_SCRATCH_BYTES = 17303552


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("x_min", ctypes.c_double),
                ("y_min", ctypes.c_double), ("dx", ctypes.c_double), ("dy", ctypes.c_double)]


class Particles(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("px", ctypes.c_void_p), ("y", ctypes.c_void_p),
                ("py", ctypes.c_void_p), ("w", ctypes.c_void_p), ("lost", ctypes.c_void_p),
                ("n", ctypes.c_int64), ("sigma", ctypes.c_void_p), ("psigma", ctypes.c_void_p)]


class Diag(ctypes.Structure):
    _fields_ = [("alive", ctypes.c_int64), ("mean", ctypes.c_double * 4),
                ("emit_x", ctypes.c_double), ("emit_y", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {"alive": int(self.alive), "mean": [float(v) for v in self.mean],
                "emit_x": float(self.emit_x), "emit_y": float(self.emit_y)}


class ScpicError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"scpic error {code}: {msg}")
        self.code = code


_lib = None


def load_library(path: Path | str | None = None):
    """Load libscpic.so (raises if it is missing)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = Path(path) if path else _LIB_PATH
    if not p.exists():
        raise RuntimeError(f"{p} is missing: build it with `python -m paper_2010_11540_amd.build`")
    L = ctypes.CDLL(str(p))
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    L.scpic_version.restype = i32
    L.scpic_last_error.restype = ctypes.c_char_p
    L.scpic_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(Grid), i32, vp]
    L.scpic_destroy.argtypes = [vp]
    L.scpic_set_stream.argtypes = [vp, vp]
    L.scpic_push.argtypes = [vp, ctypes.POINTER(Particles), vp, i32]
    L.scpic_deposit.argtypes = [vp, ctypes.POINTER(Particles), vp, vp]
    L.scpic_solve.argtypes = [vp, vp, dbl, vp, vp]
    L.scpic_kick.argtypes = [vp, ctypes.POINTER(Particles), vp, vp, dbl]
    L.scpic_track.argtypes = [vp, ctypes.POINTER(Particles), vp, i32, i32, ctypes.POINTER(Diag)]
    L.scpic_diagnose.argtypes = [vp, ctypes.POINTER(Particles), ctypes.POINTER(Diag)]
    L.scpic_set_option.argtypes = [vp, i32, i64]
    L.scpic_pass.argtypes = [vp, ctypes.POINTER(Particles), i32, dbl, vp, i32, i32]
    L.scpic_reduce_solve.argtypes = [vp, dbl]
    L.scpic_get_field.argtypes = [vp, vp, vp]
    L.scpic_set_line_density.argtypes = [vp, i32, dbl, dbl, dbl]
    L.scpic_get_line_state.argtypes = [vp, vp, vp]
    L.scpic_get_potential.argtypes = [vp, vp]
    L.scpic_batch_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(Grid),
                                     ctypes.POINTER(i64), i32, i32, vp]
    L.scpic_batch_destroy.argtypes = [vp]
    L.scpic_batch_set_stream.argtypes = [vp, vp]
    L.scpic_track_batched.argtypes = [vp, ctypes.POINTER(Particles), ctypes.POINTER(vp),
                                      ctypes.POINTER(i32), i32]
    L.scpic_batch_get_field.argtypes = [vp, i32, vp, vp]
    L.scpic_batch_autotune.argtypes = [vp, ctypes.POINTER(Particles), ctypes.POINTER(vp),
                                       ctypes.POINTER(i32), i32, ctypes.POINTER(i32),
                                       ctypes.POINTER(i32)]
    L.scpic_deposit_static.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(Particles), vp, vp,
                                       vp]
    for name in EXPORTS:
        if name not in ("scpic_version", "scpic_last_error"):
            getattr(L, name).restype = i32
    if path is None:
        _lib = L
    return L


def _check(code: int):
    if code != OK:
        raise ScpicError(code, load_library().scpic_last_error().decode())


def _stream_ptr(stream) -> int:
    s = torch.cuda.current_stream() if stream is None else stream
    return int(s.cuda_stream)


def _dev_f64(t: torch.Tensor, name: str) -> torch.Tensor:
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64
            and t.dim() == 1 and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous 1-D float64 CUDA tensor")
    return t


def particles_struct(parts: dict) -> Particles:
    x = _dev_f64(parts["x"], "x")
    n = x.shape[0]
    ptrs = []
    for k in ("x", "px", "y", "py"):
        t = _dev_f64(parts[k], k)
        if t.shape[0] != n:
            raise ValueError(f"{k} has {t.shape[0]} entries, x has {n}")
        if t.device != x.device:
            raise ValueError("particle arrays must be on one device")
        ptrs.append(t.data_ptr())
    lost = parts.get("lost")
    lp = None
    if lost is not None:
        if not (lost.is_cuda and lost.dtype == torch.uint8 and lost.is_contiguous()
                and lost.shape == (n,)):
            raise TypeError("lost must be a contiguous uint8 CUDA tensor of length n")
        lp = lost.data_ptr()
    w = parts.get("w")
    wp = None
    if w is not None:
        if not (w.is_cuda and w.dtype == torch.float32 and w.is_contiguous() and w.shape == (n,)):
            raise TypeError("w must be a contiguous float32 CUDA tensor of length n")
        wp = w.data_ptr()
    longi = []
    for k in ("sigma", "psigma"):
        t = parts.get(k)
        if t is not None:
            t = _dev_f64(t, k)
            if t.shape[0] != n or t.device != x.device:
                raise ValueError(f"{k} must have n entries on the particles' device")
            t = t.data_ptr()
        longi.append(t)
    if (longi[0] is None) != (longi[1] is None):
        raise ValueError("give both sigma and psigma, or neither")
    return Particles(*ptrs, wp, lp, n, *longi)


def _elements(elements) -> np.ndarray:
    e = np.ascontiguousarray(elements, dtype=ELEMENT_DTYPE)
    return e


def to_device(parts: dict, device="cuda") -> dict:
    """Copy a dict of numpy particle arrays to contiguous CUDA tensors."""
    out = {}
    for k, v in parts.items():
        out[k] = torch.from_numpy(np.ascontiguousarray(v)).to(device).contiguous()
    return out


def to_host(parts: dict) -> dict:
    return {k: v.cpu().numpy() for k, v in parts.items()}


def _grid_struct(grid: dict) -> Grid:
    return Grid(int(grid["nx"]), int(grid["ny"]), float(grid["x_min"]), float(grid["y_min"]),
                float(grid["dx"]), float(grid["dy"]))


def deposit_static(grid: dict, parts: dict, rho: torch.Tensor, n_in: torch.Tensor | None = None,
                   stream=None):
    """Allocation-free deposit (scpic_deposit_static) into caller-owned outputs:
    rho, a contiguous int64 CUDA tensor of nx*ny entries, and optionally n_in,
    one int64 on the same device.  Allocates nothing."""
    L = load_library()
    ncell = int(grid["nx"]) * int(grid["ny"])
    if not (isinstance(rho, torch.Tensor) and rho.is_cuda and rho.dtype == torch.int64
            and rho.is_contiguous() and rho.numel() == ncell):
        raise TypeError("rho must be a contiguous int64 CUDA tensor of nx*ny entries")
    if n_in is not None and not (n_in.is_cuda and n_in.dtype == torch.int64
                                 and n_in.numel() == 1 and n_in.device == rho.device):
        raise TypeError("n_in must be one int64 on rho's device")
    g = _grid_struct(grid)
    p = particles_struct(parts)
    _check(L.scpic_deposit_static(ctypes.byref(g), ctypes.byref(p), rho.data_ptr(),
                                  None if n_in is None else n_in.data_ptr(), _stream_ptr(stream)))


class Context:
    """One grid geometry and precision form on the current HIP device."""

    def __init__(self, grid: dict, precision: str = "fp64", stream=None):
        L = load_library()
        self._lib = L
        self.grid = dict(grid)
        self.precision = {"fp64": FP64, "mixed": MIXED}[precision]
        self.field_dtype = torch.float64 if self.precision == FP64 else torch.float32
        g = Grid(int(grid["nx"]), int(grid["ny"]), float(grid["x_min"]), float(grid["y_min"]),
                 float(grid["dx"]), float(grid["dy"]))
        h = ctypes.c_void_p()
        _check(L.scpic_create(ctypes.byref(h), ctypes.byref(g), self.precision,
                              _stream_ptr(stream)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self._lib.scpic_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _sync_stream(self, stream=None):
        _check(self._lib.scpic_set_stream(self._h, _stream_ptr(stream)))

    @property
    def ncell(self):
        return int(self.grid["nx"]) * int(self.grid["ny"])

    def set_option(self, option: int, value: int):
        _check(self._lib.scpic_set_option(self._h, option, int(value)))

    def push(self, parts: dict, elements, stream=None):
        self._sync_stream(stream)
        e = _elements(elements)
        p = particles_struct(parts)
        _check(self._lib.scpic_push(self._h, ctypes.byref(p), e.ctypes.data, len(e)))

    def deposit(self, parts: dict, stream=None):
        """(rho int64 tensor [nx*ny], n_in int64 tensor [1])"""
        self._sync_stream(stream)
        dev = parts["x"].device
        rho = torch.empty(self.ncell, dtype=torch.int64, device=dev)
        n_in = torch.empty(1, dtype=torch.int64, device=dev)
        p = particles_struct(parts)
        _check(self._lib.scpic_deposit(self._h, ctypes.byref(p), rho.data_ptr(), n_in.data_ptr()))
        return rho, n_in

    def solve(self, rho: torch.Tensor, scale: float, stream=None):
        self._sync_stream(stream)
        if not (rho.is_cuda and rho.dtype == torch.int64 and rho.is_contiguous()
                and rho.numel() == self.ncell):
            raise TypeError("rho must be a contiguous int64 CUDA tensor of nx*ny entries")
        ex = torch.empty(self.ncell, dtype=self.field_dtype, device=rho.device)
        ey = torch.empty_like(ex)
        _check(self._lib.scpic_solve(self._h, rho.data_ptr(), float(scale), ex.data_ptr(),
                                     ey.data_ptr()))
        return ex, ey

    def kick(self, parts: dict, ex: torch.Tensor, ey: torch.Tensor, kappa: float, stream=None):
        self._sync_stream(stream)
        for t in (ex, ey):
            if not (t.is_cuda and t.dtype == self.field_dtype and t.is_contiguous()
                    and t.numel() == self.ncell):
                raise TypeError(f"fields must be contiguous {self.field_dtype} CUDA tensors "
                                "of nx*ny entries")
        p = particles_struct(parts)
        _check(self._lib.scpic_kick(self._h, ctypes.byref(p), ex.data_ptr(), ey.data_ptr(),
                                    float(kappa)))

    def track(self, parts: dict, lattice, n_turns: int, stream=None, diag: bool = False):
        """Track n_turns; with diag=True return the beam diagnostics after the
        last turn (alive count, means, rms emittances; waits for the stream)."""
        self._sync_stream(stream)
        e = _elements(lattice)
        p = particles_struct(parts)
        out = Diag() if diag else None
        _check(self._lib.scpic_track(self._h, ctypes.byref(p), e.ctypes.data, len(e),
                                     int(n_turns), ctypes.byref(out) if diag else None))
        return out.as_dict() if diag else None

    def diagnose(self, parts: dict, stream=None) -> dict:
        """Alive count, means of (x, px, y, py) and rms emittances of the
        particles not lost, computed on the device; waits for the stream."""
        self._sync_stream(stream)
        p = particles_struct(parts)
        out = Diag()
        _check(self._lib.scpic_diagnose(self._h, ctypes.byref(p), ctypes.byref(out)))
        return out.as_dict()

    def pass_(self, parts: dict, kick: bool, kappa: float, elements, deposit: bool, stream=None):
        self._sync_stream(stream)
        e = _elements(elements)
        p = particles_struct(parts)
        _check(self._lib.scpic_pass(self._h, ctypes.byref(p), int(kick), float(kappa),
                                    e.ctypes.data if len(e) else None, len(e), int(deposit)))

    def reduce_solve(self, scale: float, stream=None):
        self._sync_stream(stream)
        _check(self._lib.scpic_reduce_solve(self._h, float(scale)))

    def get_field(self, stream=None):
        self._sync_stream(stream)
        dev = torch.device("cuda", torch.cuda.current_device())
        ex = torch.empty(self.ncell, dtype=self.field_dtype, device=dev)
        ey = torch.empty_like(ex)
        _check(self._lib.scpic_get_field(self._h, ex.data_ptr(), ey.data_ptr()))
        return ex, ey

    def set_line_density(self, line: dict | None, stream=None):
        """Turn the long-bunch line density on (line = {"nz", "z_min", "dz",
        "gamma0"}) or off (None)."""
        self._sync_stream(stream)
        if line is None:
            _check(self._lib.scpic_set_line_density(self._h, 0, 0.0, 1.0, 1.0))
            self.line_nz = 0
        else:
            _check(self._lib.scpic_set_line_density(self._h, int(line["nz"]), float(line["z_min"]),
                                                    float(line["dz"]), float(line["gamma0"])))
            self.line_nz = int(line["nz"])

    def get_line_state(self, stream=None):
        """(lw, ld): the line tables lambda/lambda_peak, lambda'/lambda_peak
        of the last solve (nz each)."""
        self._sync_stream(stream)
        dev = torch.device("cuda", torch.cuda.current_device())
        nz = getattr(self, "line_nz", 0)
        lw = torch.empty(max(nz, 1), dtype=torch.float64, device=dev)
        ld = torch.empty_like(lw)
        _check(self._lib.scpic_get_line_state(self._h, lw.data_ptr(), ld.data_ptr()))
        return lw[:nz], ld[:nz]

    def get_potential(self, stream=None):
        """The node potential of the last solve on nodes -1..nx by -1..ny, as
        an (nx+2, ny+2) tensor."""
        self._sync_stream(stream)
        dev = torch.device("cuda", torch.cuda.current_device())
        nx, ny = self.grid["nx"], self.grid["ny"]
        phi = torch.empty((nx + 2) * (ny + 2), dtype=self.field_dtype, device=dev)
        _check(self._lib.scpic_get_potential(self._h, phi.data_ptr()))
        return phi.reshape(nx + 2, ny + 2)


def _grid_struct(grid: dict) -> Grid:
    return Grid(int(grid["nx"]), int(grid["ny"]), float(grid["x_min"]), float(grid["y_min"]),
                float(grid["dx"]), float(grid["dy"]))


class Batch:
    """Independent beams tracked together: beam k owns particles
    offsets[k]:offsets[k+1] of the concatenated arrays and the grid grids[k]."""

    def __init__(self, grids, offsets, precision: str = "fp64", stream=None):
        L = load_library()
        self._lib = L
        self.grids = [dict(g) for g in grids]
        n = len(self.grids)
        self.offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        if self.offsets.shape != (n + 1,):
            raise ValueError(f"offsets must have {n + 1} entries")
        self.precision = {"fp64": FP64, "mixed": MIXED}[precision]
        self.field_dtype = torch.float64 if self.precision == FP64 else torch.float32
        garr = (Grid * n)(*[_grid_struct(g) for g in self.grids])
        h = ctypes.c_void_p()
        _check(L.scpic_batch_create(ctypes.byref(h), garr,
                                    self.offsets.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                    n, self.precision, _stream_ptr(stream)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self._lib.scpic_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _sync_stream(self, stream=None):
        _check(self._lib.scpic_batch_set_stream(self._h, _stream_ptr(stream)))

    def track(self, parts: dict, lattices, n_turns: int, stream=None):
        """Track every beam n_turns turns; lattices[k] is beam k's one-turn ring."""
        self._sync_stream(stream)
        els = [_elements(lat) for lat in lattices]
        if len(els) != len(self.grids):
            raise ValueError(f"need {len(self.grids)} lattices, got {len(els)}")
        ptrs = (ctypes.c_void_p * len(els))(*[e.ctypes.data for e in els])
        counts = np.array([len(e) for e in els], dtype=np.int32)
        p = particles_struct(parts)
        _check(self._lib.scpic_track_batched(
            self._h, ctypes.byref(p), ptrs,
            counts.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), int(n_turns)))

    def autotune(self, parts: dict, lattices, trial_turns: int = 2, stream=None):
        """Time the candidate pass shapes on a scratch copy of parts and keep the
        fastest; returns (threads per workgroup, workgroups per compute unit)."""
        self._sync_stream(stream)
        els = [_elements(lat) for lat in lattices]
        ptrs = (ctypes.c_void_p * len(els))(*[e.ctypes.data for e in els])
        counts = np.array([len(e) for e in els], dtype=np.int32)
        p = particles_struct(parts)
        t = ctypes.c_int32()
        c = ctypes.c_int32()
        _check(self._lib.scpic_batch_autotune(
            self._h, ctypes.byref(p), ptrs,
            counts.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), int(trial_turns),
            ctypes.byref(t), ctypes.byref(c)))
        return t.value, c.value

    def get_field(self, k: int, stream=None):
        self._sync_stream(stream)
        g = self.grids[k]
        ncell = int(g["nx"]) * int(g["ny"])
        dev = torch.device("cuda", torch.cuda.current_device())
        ex = torch.empty(ncell, dtype=self.field_dtype, device=dev)
        ey = torch.empty_like(ex)
        _check(self._lib.scpic_batch_get_field(self._h, int(k), ex.data_ptr(), ey.data_ptr()))
        return ex, ey
