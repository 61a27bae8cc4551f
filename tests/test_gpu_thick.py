"""Six-dimensional tracking through thick elements on the HIP path (chromatic
thick quadrupole, Sec. III-B; thick sextupole by the symmetric split of
Sec. III-C), through the C ABI, against the FP64 CPU oracle.

Bars:
  push through thick elements   max|u - u_ref| / rms(u_ref) <= 1e-12 per coordinate
                                (both sides FP64: they differ only in the rounding
                                of sin/cos/cosh/sinh and in the algebraic form of
                                the path-length integral, a few ulp per element)
  one turn with space charge    <= 1e-10 per coordinate (FP64); the FP32 field bar
                                over the turn's kicks (mixed)
  batched == single-beam path   bit-exact
"""
import sys

import numpy as np
import pytest

from paper_2010_11540_amd import inputs

pytestmark = pytest.mark.gpu

COORDS6 = ("x", "px", "y", "py", "sigma", "psigma")
IG2 = 1.0 / inputs.GAMMA0_3GEV ** 2


def _say(msg):
    print(f"\n[case] {msg}", flush=True)
    sys.stdout.flush()


def _dev(parts):
    from paper_2010_11540_amd.scpic import to_device
    return to_device(parts)


def _host(parts):
    return {k: v.cpu().numpy() for k, v in parts.items()}


def _err6(h, ref):
    if ref["x"].shape[0] == 0:
        return 0.0
    return max(np.abs(h[k] - ref[k]).max() / max(ref[k].std(), 1e-300) for k in COORDS6)


def _mixed_bar(orc, w, ref):
    """The FP32 field bar (1e-5 of max|E|) over every kick of the turn,
    relative to the rms momenta."""
    q, _ = orc.deposit(inputs.copy_parts(w["parts"]), w["grid"])
    ex0, ey0 = orc.solve(q, 1.0 / ((1 << 24) * w["n"]), w["grid"])
    lat = w["lattice"]
    kappa = float(lat["p"][lat["kind"] == inputs.SC][0, 0])
    n_sc = int((lat["kind"] == inputs.SC).sum())
    emax = max(np.abs(ex0).max(), np.abs(ey0).max())
    return 2 * n_sc * 1e-5 * kappa * emax / min(ref["px"].std(), ref["py"].std())


def _thick_mix():
    """Every thick form: focusing, defocusing and zero-gradient quadrupoles,
    sextupoles of both signs with 1, 3 and 17 split steps, a drift, and the
    four-dimensional kinds in between (16 elements: two passes)."""
    return np.concatenate([
        inputs.quad_thick(0.9, 0.4, IG2), inputs.drift(1.1, IG2),
        inputs.sext_thick(40.0, 0.3, IG2, 1), inputs.quad_thick(-1.2, 0.5, IG2),
        inputs.sext_thick(-25.0, 0.2, IG2, 3), inputs.quad_thick(0.0, 0.7, IG2),
        inputs.lin2x2(inputs.rotation(0.7), inputs.rotation(1.1)),
        inputs.sext_thin(3.0), inputs.sext_thick(60.0, 0.25, IG2, 17),
        inputs.quad_thick(0.3, 1.5, IG2), inputs.lin4x4(inputs.random_symplectic4(5)),
        inputs.drift(-0.4, IG2), inputs.quad_thick(-0.05, 2.0, IG2),
        inputs.sext_thick(0.0, 0.6, IG2, 2), inputs.quad_thick(2.5, 0.3, IG2),
        inputs.drift(0.9, IG2)])


@pytest.mark.parametrize("case,n", [("mix", 10_007), ("mix", 1), ("mix", 300_001),
                                    ("fodo", 100_003), ("wide", 50_001)])
def test_thick_push_matches_oracle(gpu, orc, case, n):
    """mix: one push through every thick form (the mix is not a stable ring:
    one pass only); fodo: three turns of the thick FODO ring with 3-step
    sextupoles; wide: the mix with a momentum spread (p_sigma rms 0.15) so wide
    that many particles' quadrupole angles differ from the on-momentum angle
    by more than 1/16 rad, the limit of the kernel's short-series path."""
    _say(f"push {n} particles through {case}")
    if case in ("mix", "wide"):
        lat, reps = _thick_mix(), 1
    else:
        lat, reps = inputs.fodo_thick(16, 4.2, None, sext_steps=3), 3
    p0 = inputs.gaussian_beam6d(n, 40 + n, sigma_ps=0.15 if case == "wide" else 3e-3)
    if case == "wide":
        quads = lat[lat["kind"] == inputs.QUAD_THICK]
        phi0 = np.sqrt(np.abs(quads["p"][:, 0])) * quads["p"][:, 1]
        d = np.abs(phi0[:, None] * (np.sqrt(1.0 - p0["psigma"][None, :]) - 1.0))
        assert (d > 1 / 16).mean() > 0.05 and (d <= 1 / 16).mean() > 0.5
    ref = inputs.copy_parts(p0)
    for _ in range(reps):
        orc.push(ref, lat)
    assert all(np.isfinite(ref[k]).all() for k in COORDS6)
    with gpu.Context(inputs.make_grid(64)) as ctx:
        d = _dev(p0)
        for _ in range(reps):
            ctx.push(d, lat)
        h = _host(d)
    np.testing.assert_array_equal(h["psigma"], p0["psigma"])
    err = _err6(h, ref) if n > 1 else max(
        np.abs(h[k] - ref[k]).max() / (1.0 if k == "sigma" else 1e-3) for k in COORDS6)
    print(f"[thick push] {case} n={n} max error {err:.3e} of rms", flush=True)
    assert err <= 1e-12, err


@pytest.mark.parametrize("use_graph", [True, False])
def test_thick_small_one_turn_fp64(gpu, orc, use_graph):
    _say(f"thick_small workload 1 turn fp64 (graph={use_graph})")
    w = inputs.workload("thick_small")
    ref = inputs.copy_parts(w["parts"])
    orc.track(ref, w["grid"], w["lattice"], 1)
    with gpu.Context(w["grid"]) as ctx:
        ctx.set_option(gpu.OPT_USE_GRAPH, int(use_graph))
        d = _dev(w["parts"])
        ctx.track(d, w["lattice"], 1)
        h = _host(d)
    np.testing.assert_array_equal(h["lost"], ref["lost"])
    err = _err6(h, ref)
    print(f"[thick small] one-turn error {err:.3e} of rms", flush=True)
    assert err <= 1e-10, err


def test_thick_small_one_turn_mixed(gpu, orc):
    _say("thick_small workload 1 turn mixed")
    w = inputs.workload("thick_small")
    ref = inputs.copy_parts(w["parts"])
    orc.track(ref, w["grid"], w["lattice"], 1)
    with gpu.Context(w["grid"], "mixed") as ctx:
        d = _dev(w["parts"])
        ctx.track(d, w["lattice"], 1)
        h = _host(d)
    np.testing.assert_array_equal(h["lost"], ref["lost"])
    err = _err6(h, ref)
    bar = _mixed_bar(orc, w, ref)
    print(f"[thick small mixed] one-turn error {err:.3e} (bar {bar:.3e})", flush=True)
    assert err <= bar, (err, bar)


@pytest.fixture(scope="module")
def thick_one_turn_reference(orc):
    w = inputs.workload("thick")
    ref = inputs.copy_parts(w["parts"])
    orc.track(ref, w["grid"], w["lattice"], 1)
    return w, ref


def test_thick_workload_full_size_one_turn_fp64(gpu, thick_one_turn_reference):
    """The 6D thick workload at full size (1e6 particles, 128^2, 100 FODO cells
    of thick quadrupoles and sextupoles, 100 SC steps) in the launch
    configuration the benchmark times."""
    _say("thick workload full size 1 turn fp64 (1e6 particles)")
    w, ref = thick_one_turn_reference
    with gpu.Context(w["grid"]) as ctx:
        d = _dev(w["parts"])
        ctx.track(d, w["lattice"], 1)
        h = _host(d)
    np.testing.assert_array_equal(h["lost"], ref["lost"])
    err = _err6(h, ref)
    print(f"[thick full] one-turn error {err:.3e} of rms", flush=True)
    assert err <= 1e-10, err


def test_thick_elements_reject_missing_longitudinal_arrays(gpu):
    _say("thick element argument checks")
    p0 = inputs.gaussian_beam6d(1000, 9)
    four = {k: v for k, v in p0.items() if k not in ("sigma", "psigma")}
    with gpu.Context(inputs.make_grid(32)) as ctx:
        d = _dev(four)
        for lat in (inputs.quad_thick(1.0, 0.5, IG2), inputs.fodo_thick(4, 1.1, 1e-9)):
            with pytest.raises(gpu.ScpicError) as e:
                ctx.track(d, lat, 1)
            assert e.value.code == gpu.EINVAL
        with pytest.raises(gpu.ScpicError) as e:
            ctx.push(d, inputs.sext_thick(1.0, 0.5, IG2, 1))
        assert e.value.code == gpu.EINVAL
        d6 = _dev(p0)
        for steps in (0, 1025):
            bad = inputs.sext_thick(1.0, 0.5, IG2, 1)
            bad["p"][0, 3] = steps
            with pytest.raises(gpu.ScpicError) as e:
                ctx.push(d6, bad)
            assert e.value.code == gpu.EINVAL
        bad = inputs.quad_thick(1.0, 0.5, IG2)
        bad["p"][0, 1] = np.inf
        with pytest.raises(gpu.ScpicError) as e:
            ctx.track(d6, bad, 1)
        assert e.value.code == gpu.EINVAL
        h = _host(d6)
    for k in COORDS6:
        np.testing.assert_array_equal(h[k], p0[k])


def test_four_dimensional_lattice_leaves_longitudinal_alone(gpu):
    _say("small workload lattice with 6D particles == 4D run, sigma untouched")
    w = inputs.workload("small")
    p6 = inputs.gaussian_beam6d(w["n"], 77)
    p4 = {k: v for k, v in p6.items() if k not in ("sigma", "psigma")}
    outs = []
    with gpu.Context(w["grid"]) as ctx:
        for p in (p6, p4):
            d = _dev(p)
            ctx.track(d, w["lattice"], 2)
            outs.append(_host(d))
    for k in ("x", "px", "y", "py", "lost"):
        np.testing.assert_array_equal(outs[0][k], outs[1][k])
    np.testing.assert_array_equal(outs[0]["sigma"], p6["sigma"])
    np.testing.assert_array_equal(outs[0]["psigma"], p6["psigma"])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_of_thick_rings_equals_single_beam(gpu, precision):
    """Four beams, three on thick FODO rings of different tunes and one on a
    four-dimensional ring with the same 16 SC locations: the batched passes
    run the six-dimensional kernels for all, and every beam equals its
    single-beam run bit for bit."""
    _say(f"batch of thick rings, 3 turns, {precision}")
    eps = 1e-6 / inputs.fodo_beta(16, 4.2)[0]
    kappa = inputs.kappa_for_tune_shift(-0.2, eps, 16)
    lattices = [inputs.fodo_thick(16, 4.2, kappa), inputs.fodo_thick(16, 4.05, kappa, sext_steps=2),
                inputs.ring(4.2, 4.3, 16, inputs.kappa_for_tune_shift(-0.2, 1e-6, 16)),
                inputs.fodo_thick(16, 4.3, 2 * kappa, k2f=0.0, k2d=0.0)]
    grids = [inputs.make_grid(64), inputs.make_grid(32), inputs.make_grid(64), inputs.make_grid(64, 32)]
    bx, by = inputs.fodo_beta(16, 4.2)
    sizes = [5000, 777, 12000, 3000]
    beams = []
    for k, n in enumerate(sizes):
        if k == 2:
            beams.append(inputs.gaussian_beam6d(n, 900 + k))
        else:
            beams.append(inputs.gaussian_beam6d(n, 900 + k, 1e-3, 1e-3 / bx, 1e-3 * (by / bx) ** 0.5,
                                                1e-3 / (bx * by) ** 0.5))
    parts, offsets = inputs.concat_parts(beams)
    with gpu.Batch(grids, offsets, precision) as b:
        d = _dev(parts)
        b.track(d, lattices, 3)
        got = _host(d)
    for k in range(len(sizes)):
        a, z = int(offsets[k]), int(offsets[k + 1])
        with gpu.Context(grids[k], precision) as ctx:
            dk = _dev({key: v[a:z].copy() for key, v in parts.items()})
            ctx.track(dk, lattices[k], 3)
            want = _host(dk)
        for key in COORDS6 + ("lost",):
            np.testing.assert_array_equal(got[key][a:z], want[key], err_msg=f"beam {k} {key}")
