"""CPU-side checks of the C ABI: the library loads, exports every function
include/scpic.h declares, and rejects invalid arguments before touching any
GPU state (no compute calls)."""
import ctypes
import re
from pathlib import Path

import numpy as np
import pytest

ROOT = Path(__file__).resolve().parent.parent
HEADER = ROOT / "include" / "scpic.h"
LIB = ROOT / "paper_2010_11540_amd" / "libscpic.so"


def _declared_functions():
    text = HEADER.read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(scpic_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not LIB.exists():
        from paper_2010_11540_amd import build
        build.build()
    from paper_2010_11540_amd import scpic
    return scpic.load_library(LIB)


def test_header_declares_the_binding_exports():
    from paper_2010_11540_amd import scpic
    assert _declared_functions() == sorted(scpic.EXPORTS)


def test_every_declared_symbol_is_exported(lib):
    for name in _declared_functions():
        assert hasattr(lib, name), name


def test_version_and_empty_error(lib):
    assert lib.scpic_version() >= 100
    assert isinstance(lib.scpic_last_error(), bytes)


def test_element_layout_matches_header():
    from paper_2010_11540_amd import inputs
    assert inputs.ELEMENT_DTYPE.itemsize == 136
    assert inputs.ELEMENT_DTYPE.fields["p"][1] == 8


def _grid(nx=64, ny=64, dx=1e-4, dy=1e-4):
    from paper_2010_11540_amd.scpic import Grid
    return Grid(nx, ny, -3e-3, -3e-3, dx, dy)


@pytest.mark.parametrize("kw,code", [({"ny": 102}, -4), ({"ny": 512}, -4), ({"nx": 4}, -4),
                                     ({"nx": 257}, -4), ({"ny": 260}, -4), ({"ny": 4}, -4),
                                     ({"dx": 0.0}, -1), ({"dy": -1e-4}, -1),
                                     ({"dx": float("nan")}, -1), ({"nx": 512, "ny": 256}, -4)])
def test_create_rejects_bad_grids_before_touching_the_device(lib, kw, code):
    h = ctypes.c_void_p(123)
    g = _grid(**kw)
    assert lib.scpic_create(ctypes.byref(h), ctypes.byref(g), 0, None) == code
    assert h.value is None
    assert lib.scpic_last_error()


def test_create_rejects_null_and_bad_precision(lib):
    h = ctypes.c_void_p()
    g = _grid()
    assert lib.scpic_create(None, ctypes.byref(g), 0, None) == -1
    assert lib.scpic_create(ctypes.byref(h), None, 0, None) == -1
    assert lib.scpic_create(ctypes.byref(h), ctypes.byref(g), 7, None) == -1


def test_calls_on_null_context_are_einval(lib):
    from paper_2010_11540_amd.scpic import Particles
    p = Particles(None, None, None, None, None, None, 0)
    e = np.zeros(1, dtype=[("kind", "<i4"), ("pad", "<i4"), ("p", "<f8", (16,))])
    assert lib.scpic_destroy(None) == 0
    assert lib.scpic_push(None, ctypes.byref(p), e.ctypes.data, 1) == -1
    assert lib.scpic_deposit(None, ctypes.byref(p), None, None) == -1
    assert lib.scpic_solve(None, None, 1.0, None, None) == -1
    assert lib.scpic_kick(None, ctypes.byref(p), None, None, 1.0) == -1
    assert lib.scpic_track(None, ctypes.byref(p), e.ctypes.data, 1, 1, None) == -1
    assert lib.scpic_diagnose(None, ctypes.byref(p), None) == -1
    assert lib.scpic_set_option(None, 1, 1) == -1
    assert lib.scpic_set_option(None, 4, 1) == -1
    assert lib.scpic_set_stream(None, None) == -1
    assert lib.scpic_pass(None, ctypes.byref(p), 0, 0.0, None, 0, 0) == -1
    assert lib.scpic_reduce_solve(None, 1.0) == -1
    assert lib.scpic_get_field(None, None, None) == -1
    assert b"ctx" in lib.scpic_last_error()


def test_batch_create_rejects_bad_arguments_before_touching_the_device(lib):
    from paper_2010_11540_amd.scpic import Grid
    h = ctypes.c_void_p(123)
    good = (Grid * 2)(_grid(), _grid(32, 32))
    bad_grid = (Grid * 2)(_grid(), _grid(ny=98))
    off = lambda *v: (ctypes.c_int64 * len(v))(*v)
    cases = [
        (good, off(0, 10, 20), 0, 0, -1),     # n_inst 0
        (good, off(1, 10, 20), 2, 0, -1),     # offsets[0] != 0
        (good, off(0, 10, 5), 2, 0, -1),      # decreasing
        (good, off(0, 10, 20), 2, 5, -1),     # precision
        (bad_grid, off(0, 10, 20), 2, 0, -4),  # grid limits
    ]
    for grids, offs, n, prec, code in cases:
        assert lib.scpic_batch_create(ctypes.byref(h), grids, offs, n, prec, None) == code
        assert h.value is None
        assert lib.scpic_last_error()
    assert lib.scpic_batch_create(None, good, off(0, 1, 2), 2, 0, None) == -1
    assert lib.scpic_batch_create(ctypes.byref(h), None, off(0, 1, 2), 2, 0, None) == -1
    assert lib.scpic_batch_create(ctypes.byref(h), good, None, 2, 0, None) == -1


def test_batch_calls_on_null_batch_are_einval(lib):
    from paper_2010_11540_amd.scpic import Particles
    p = Particles(None, None, None, None, None, None, 0)
    assert lib.scpic_batch_destroy(None) == 0
    assert lib.scpic_batch_set_stream(None, None) == -1
    assert lib.scpic_track_batched(None, ctypes.byref(p), None, None, 1) == -1
    assert lib.scpic_batch_get_field(None, 0, None, None) == -1
    assert lib.scpic_batch_autotune(None, ctypes.byref(p), None, None, 1, None, None) == -1
    assert b"batch" in lib.scpic_last_error()


def test_static_deposit_rejects_bad_arguments_before_touching_the_device(lib):
    from paper_2010_11540_amd.scpic import Particles
    p = Particles(None, None, None, None, None, None, 0)
    neg = Particles(None, None, None, None, None, None, -1)
    nulls = Particles(None, None, None, None, None, None, 5)
    rho = ctypes.c_void_p(0x1000)
    g = _grid()
    assert lib.scpic_deposit_static(None, ctypes.byref(p), rho, None, None) == -1
    assert lib.scpic_deposit_static(ctypes.byref(g), None, rho, None, None) == -1
    assert lib.scpic_deposit_static(ctypes.byref(g), ctypes.byref(p), None, None, None) == -1
    assert lib.scpic_deposit_static(ctypes.byref(g), ctypes.byref(neg), rho, None, None) == -1
    assert lib.scpic_deposit_static(ctypes.byref(g), ctypes.byref(nulls), rho, None, None) == -1
    for kw, code in (({"nx": 257}, -4), ({"ny": 102}, -4), ({"dx": 0.0}, -1)):
        bad = _grid(**kw)
        assert lib.scpic_deposit_static(ctypes.byref(bad), ctypes.byref(p), rho, None, None) == code
        assert lib.scpic_last_error()


def test_static_scratch_size_matches_the_header():
    from paper_2010_11540_amd import scpic
    text = HEADER.read_text()
    m = re.search(r"#define SCPIC_STATIC_SCRATCH_BYTES (\d+)", text)
    assert m and int(m.group(1)) == scpic.STATIC_SCRATCH_BYTES
    # 64 workgroups' uint32 partials of a 65536-node grid, their 32-byte
    # headers and a uint64 carry grid of 65536 nodes
    assert scpic.STATIC_SCRATCH_BYTES == 64 * 65536 * 4 + 64 * 32 + 65536 * 8
