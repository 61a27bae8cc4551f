"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Bars:
  deposit            bit-exact (integer charge grid, lost flags, count)
  push               bit-exact (both sides evaluate the same IEEE sums, no FMA)
  kick (same field)  bit-exact in FP64
  solve              max|E - E_ref| / max|E_ref| <= 1e-12 (FP64), 1e-5 (FP32)
  one turn           max|u - u_ref| / rms(u_ref) <= 1e-10 per coordinate (FP64)
"""
import math
import sys

import numpy as np
import pytest

from paper_2010_11540_amd import inputs

pytestmark = pytest.mark.gpu

COORDS = ("x", "px", "y", "py")


def _say(msg):
    print(f"\n[case] {msg}", flush=True)
    sys.stdout.flush()


def _dev(parts):
    from paper_2010_11540_amd.scpic import to_device
    return to_device(parts)


def _host(parts):
    return {k: v.cpu().numpy() for k, v in parts.items()}


def _field_err(got, want):
    return np.abs(got - want).max() / np.abs(want).max()


# ------------------------------------------------------------------ deposit

@pytest.mark.parametrize("n,nx,ny,seed", [(10_000, 64, 64, 1), (1, 64, 64, 2), (63, 32, 16, 3),
                                          (100_003, 128, 128, 4), (0, 64, 64, 5),
                                          (1_000_000, 128, 128, 6), (257_000, 64, 128, 7),
                                          (100_000, 100, 100, 21), (257_003, 96, 64, 22),
                                          (50_001, 37, 100, 23), (1_000_000, 100, 100, 24)])
def test_deposit_bit_exact(gpu, orc, n, nx, ny, seed):
    _say(f"deposit n={n} grid={nx}x{ny} seed={seed}")
    g = inputs.make_grid(nx, ny, 4.5e-3, 5e-3)
    p = inputs.gaussian_beam(n, seed)
    ref = inputs.copy_parts(p)
    q_ref, n_ref = orc.deposit(ref, g)
    with gpu.Context(g) as ctx:
        d = _dev(p)
        rho, n_in = ctx.deposit(d)
        np.testing.assert_array_equal(rho.cpu().numpy(), q_ref)
        assert int(n_in.item()) == n_ref
        np.testing.assert_array_equal(d["lost"].cpu().numpy(), ref["lost"])


@pytest.mark.parametrize("kind,n,nx,ny", [("kv", 1_000_003, 256, 256), ("box", 300_001, 256, 256),
                                         ("box", 200_000, 256, 64), ("box", 150_000, 128, 128)])
def test_deposit_bit_exact_large_grids_and_wide_beams(gpu, orc, kind, n, nx, ny):
    """256-node grids (larger than one workgroup's LDS) and beams spanning the
    whole grid: cells outside a workgroup's LDS tile take the global path."""
    _say(f"deposit large grid kind={kind} n={n} grid={nx}x{ny}")
    g = inputs.make_grid(nx, ny, 12e-3, 6e-3)
    p = inputs.long_bunch_kv(n, 17) if kind == "kv" else inputs.uniform_in_box(n, 18, g)
    ref = inputs.copy_parts(p)
    q_ref, n_ref = orc.deposit(ref, g)
    with gpu.Context(g) as ctx:
        d = _dev(p)
        for rep in range(3):  # later calls reuse the previous boxes as tiles
            rho, n_in = ctx.deposit(d)
            np.testing.assert_array_equal(rho.cpu().numpy(), q_ref)
            assert int(n_in.item()) == n_ref


def test_deposit_overflow_path_all_on_one_node(gpu, orc):
    """2^18 particles on one node: every LDS cell of every workgroup wraps
    2^32 many times; the carries must restore the exact 2^42 total."""
    _say("deposit overflow: 262144 particles on one node")
    g = inputs.make_grid(64)
    n = 1 << 18
    p = {"x": np.full(n, g["x_min"] + 17 * g["dx"]), "px": np.zeros(n),
         "y": np.full(n, g["y_min"] + 40 * g["dy"]), "py": np.zeros(n),
         "lost": np.zeros(n, dtype=np.uint8)}
    q_ref, _ = orc.deposit(inputs.copy_parts(p), g)
    with gpu.Context(g) as ctx:
        rho, n_in = ctx.deposit(_dev(p))
        got = rho.cpu().numpy()
    np.testing.assert_array_equal(got, q_ref)
    assert got.reshape(64, 64)[17, 40] == n << 24


def test_deposit_edges_nan_inf_and_lost(gpu, orc):
    _say("deposit edges / NaN / inf / pre-lost")
    g = inputs.make_grid(16)
    top = g["x_min"] + 15 * g["dx"]
    xs = np.array([g["x_min"], top, top - 1e-6 * g["dx"], np.nan, 0.0, np.inf, -np.inf, 0.0,
                   1e-3, 2e-3])
    ys = np.array([0.0, 0.0, 0.0, 0.0, np.nan, 0.0, 0.0, g["y_min"] - 1e-12, 1e-3, -2e-3])
    p = {"x": xs, "px": np.zeros(10), "y": ys, "py": np.zeros(10),
         "lost": np.zeros(10, dtype=np.uint8)}
    p["lost"][9] = 1
    ref = inputs.copy_parts(p)
    q_ref, n_ref = orc.deposit(ref, g)
    with gpu.Context(g) as ctx:
        d = _dev(p)
        rho, n_in = ctx.deposit(d)
        np.testing.assert_array_equal(rho.cpu().numpy(), q_ref)
        np.testing.assert_array_equal(d["lost"].cpu().numpy(), ref["lost"])
        assert int(n_in.item()) == n_ref == 3


@pytest.mark.parametrize("threads,blocks", [(256, 0), (512, 7), (1024, 1), (1024, 0), (256, 3)])
def test_deposit_independent_of_launch_shape_and_repeatable(gpu, orc, threads, blocks):
    _say(f"deposit launch shape threads={threads} blocks={blocks}")
    g = inputs.make_grid(128)
    p = inputs.gaussian_beam(300_001, 11)
    q_ref, _ = orc.deposit(inputs.copy_parts(p), g)
    with gpu.Context(g) as ctx:
        ctx.set_option(gpu.OPT_PASS_THREADS, threads)
        ctx.set_option(gpu.OPT_PASS_BLOCKS, blocks)
        d = _dev(p)
        r1, _ = ctx.deposit(d)
        r2, _ = ctx.deposit(d)
        np.testing.assert_array_equal(r1.cpu().numpy(), q_ref)
        np.testing.assert_array_equal(r2.cpu().numpy(), q_ref)


# --------------------------------------------------------------------- push

def test_push_bit_exact(gpu, orc):
    _say("push: 2x2, 4x4 coupled, sextupoles, > 12 elements")
    p = inputs.gaussian_beam(70_001, 12)
    p["lost"][::7] = 1
    lat = np.concatenate([inputs.ring(4.2, 4.3, 16, kappa=None),
                          inputs.ring(4.2, 4.3, 5, kappa=None, four_by_four=True, k2l=5.0,
                                      sext_every=2, coupled=inputs.random_symplectic4(3)),
                          inputs.sc_kick(1.0)])
    assert len(lat) > 12
    ref = inputs.copy_parts(p)
    orc.push(ref, lat)
    with gpu.Context(inputs.make_grid(64)) as ctx:
        d = _dev(p)
        ctx.push(d, lat)
        h = _host(d)
    for k in COORDS:
        np.testing.assert_array_equal(h[k], ref[k])


# --------------------------------------------------------------------- solve

def _charge(n, seed, g, orc):
    p = inputs.gaussian_beam(n, seed, sigma_x=1.1e-3, sigma_y=0.8e-3)
    q, n_in = orc.deposit(p, g)
    return q, 1.0 / ((1 << 24) * n)


@pytest.mark.parametrize("nx,ny,hx,hy", [(64, 64, 6e-3, 6e-3), (128, 128, 6e-3, 6e-3),
                                         (64, 32, 6e-3, 4e-3), (16, 128, 5e-3, 7e-3),
                                         (8, 8, 6e-3, 6e-3), (256, 256, 12e-3, 6e-3),
                                         (256, 32, 8e-3, 3e-3),
                                         # not powers of two: padded to the next power
                                         # of two of at least twice the side
                                         (100, 100, 6e-3, 6e-3), (96, 64, 6e-3, 4e-3),
                                         (37, 100, 3e-3, 7e-3), (200, 36, 8e-3, 3e-3),
                                         (9, 12, 2e-3, 2e-3)])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("mixed", 1e-5)])
def test_solve_matches_oracle(gpu, orc, nx, ny, hx, hy, precision, tol):
    _say(f"solve {precision} grid={nx}x{ny}")
    g = inputs.make_grid(nx, ny, hx, hy)
    q, scale = _charge(50_000, 13, g, orc)
    ex_ref, ey_ref = orc.solve(q, scale, g)
    import torch
    with gpu.Context(g, precision) as ctx:
        ex, ey = ctx.solve(torch.from_numpy(q).cuda(), scale)
        ex = ex.double().cpu().numpy()
        ey = ey.double().cpu().numpy()
    assert _field_err(ex, ex_ref) <= tol, _field_err(ex, ex_ref)
    assert _field_err(ey, ey_ref) <= tol, _field_err(ey, ey_ref)


@pytest.mark.parametrize("nx,ny,hx,hy", [(32, 16, 4e-3, 3e-3), (64, 64, 6e-3, 6e-3),
                                         (128, 128, 6e-3, 6e-3), (16, 128, 5e-3, 7e-3),
                                         (256, 256, 12e-3, 6e-3)])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("mixed", 1e-5)])
def test_pipe_solve_matches_oracle(gpu, orc, nx, ny, hx, hy, precision, tol):
    _say(f"pipe solve {precision} grid={nx}x{ny}")
    g = inputs.make_grid(nx, ny, hx, hy)
    q, scale = _charge(50_000, 17, g, orc)
    ex_ref, ey_ref = orc.solve(q, scale, g, "pipe")
    import torch
    with gpu.Context(g, precision) as ctx:
        ctx.set_option(gpu.OPT_SOLVER, gpu.SOLVER_PIPE)
        ex, ey = ctx.solve(torch.from_numpy(q).cuda(), scale)
        ex = ex.double().cpu().numpy()
        ey = ey.double().cpu().numpy()
    assert _field_err(ex, ex_ref) <= tol, _field_err(ex, ex_ref)
    assert _field_err(ey, ey_ref) <= tol, _field_err(ey, ey_ref)


def test_pipe_needs_power_of_two_sides(gpu):
    _say("pipe rejects a 100 x 100 grid")
    g = inputs.make_grid(100, 100, 6e-3, 6e-3)
    with gpu.Context(g) as ctx:
        with pytest.raises(gpu.ScpicError) as e:
            ctx.set_option(gpu.OPT_SOLVER, gpu.SOLVER_PIPE)
        assert e.value.code == -4


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_one_turn_on_the_papers_100_grid(gpu, orc, precision):
    """The small ring on a 100 x 100 grid over +-6 sigma (the paper's grid
    size): one turn of 16 SC steps, graph on, against the oracle."""
    _say(f"track 100x100 grid 1 turn {precision}")
    g = inputs.make_grid(100)
    p = inputs.gaussian_beam(20_011, 31)
    lat = inputs.ring(4.2, 4.3, 16, inputs.kappa_for_tune_shift(-0.2, 1e-6, 16))
    ref = inputs.copy_parts(p)
    orc.track(ref, g, lat, 1)
    with gpu.Context(g, precision) as ctx:
        d = _dev(p)
        ctx.track(d, lat, 1)
        h = _host(d)
    np.testing.assert_array_equal(h["lost"], ref["lost"])
    err = _turn_err(h, ref)
    bar = 1e-10
    if precision == "mixed":
        # each of the 16 kicks carries at most the FP32 field bar (1e-5 of
        # max|E|) times kappa, relative to the rms momenta, doubled
        q, _ = orc.deposit(inputs.copy_parts(p), g)
        ex0, ey0 = orc.solve(q, 1.0 / ((1 << 24) * len(p["x"])), g)
        kappa = float(lat["p"][lat["kind"] == inputs.SC][0, 0])
        emax = max(np.abs(ex0).max(), np.abs(ey0).max())
        bar = 2 * 16 * 1e-5 * kappa * emax / min(ref["px"].std(), ref["py"].std())
    print(f"[result] 100x100 one turn {precision}: {err:.3e} (bar {bar:.3e})", flush=True)
    assert err <= bar, (err, bar)


def test_solve_zero_charge_gives_zero_field(gpu):
    _say("solve zero charge")
    import torch
    g = inputs.make_grid(32)
    with gpu.Context(g) as ctx:
        ex, ey = ctx.solve(torch.zeros(32 * 32, dtype=torch.int64, device="cuda"), 1.0)
        assert float(ex.abs().max()) == 0.0 and float(ey.abs().max()) == 0.0


# ---------------------------------------------------------------------- kick

@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_kick_with_oracle_field(gpu, orc, precision):
    _say(f"kick {precision}")
    import torch
    g = inputs.make_grid(64)
    p = inputs.gaussian_beam(100_001, 14)
    q, scale = _charge(100_001, 14, g, orc)
    ex_ref, ey_ref = orc.solve(q, scale, g)
    ref = inputs.copy_parts(p)
    kappa = 5.0e-8
    orc.kick(ref, g, ex_ref, ey_ref, kappa)
    fdt = torch.float64 if precision == "fp64" else torch.float32
    with gpu.Context(g, precision) as ctx:
        d = _dev(p)
        ctx.kick(d, torch.from_numpy(ex_ref).to("cuda", fdt), torch.from_numpy(ey_ref).to("cuda", fdt),
                 kappa)
        h = _host(d)
    np.testing.assert_array_equal(h["lost"], ref["lost"])
    for k in ("x", "y"):
        np.testing.assert_array_equal(h[k], ref[k])
    for k in ("px", "py"):
        if precision == "fp64":
            np.testing.assert_array_equal(h[k], ref[k])
        else:
            dk = np.abs((h[k] - p[k]) - (ref[k] - p[k])).max()
            assert dk <= 1e-5 * np.abs(ref[k] - p[k]).max()


# ---------------------------------------------------------------- full loop

def _turn_err(h, ref):
    return max(np.abs(h[k] - ref[k]).max() / ref[k].std() for k in COORDS)


@pytest.mark.parametrize("use_graph", [True, False])
def test_small_workload_one_turn_fp64(gpu, orc, use_graph):
    _say(f"track small workload 1 turn fp64 graph={use_graph}")
    w = inputs.workload("small")
    ref = inputs.copy_parts(w["parts"])
    orc.track(ref, w["grid"], w["lattice"], 1)
    with gpu.Context(w["grid"]) as ctx:
        ctx.set_option(gpu.OPT_USE_GRAPH, int(use_graph))
        d = _dev(w["parts"])
        ctx.track(d, w["lattice"], 1)
        h = _host(d)
    np.testing.assert_array_equal(h["lost"], ref["lost"])
    assert _turn_err(h, ref) <= 1e-10, _turn_err(h, ref)


@pytest.mark.parametrize("use_graph", [True, False])
def test_small_workload_one_turn_pipe_fp64(gpu, orc, use_graph):
    """The small workload in a grounded pipe (walls at the grid's first node
    and one spacing past its last) against the oracle; switching back to the
    open boundary then reproduces the open-boundary turn."""
    _say(f"track small workload 1 turn, grounded pipe, graph={use_graph}")
    w = inputs.workload("small")
    ref = inputs.copy_parts(w["parts"])
    orc.track(ref, w["grid"], w["lattice"], 1, solver="pipe")
    ref_open = inputs.copy_parts(w["parts"])
    orc.track(ref_open, w["grid"], w["lattice"], 1)
    with gpu.Context(w["grid"]) as ctx:
        ctx.set_option(gpu.OPT_USE_GRAPH, int(use_graph))
        d = _dev(w["parts"])
        ctx.track(d, w["lattice"], 1)  # open boundary first: caches its turn
        ctx.set_option(gpu.OPT_SOLVER, gpu.SOLVER_PIPE)
        d = _dev(w["parts"])
        ctx.track(d, w["lattice"], 1)
        h = _host(d)
        ctx.set_option(gpu.OPT_SOLVER, gpu.SOLVER_OPEN)
        d = _dev(w["parts"])
        ctx.track(d, w["lattice"], 1)
        h_open = _host(d)
    np.testing.assert_array_equal(h["lost"], ref["lost"])
    assert _turn_err(h, ref) <= 1e-10, _turn_err(h, ref)
    assert _turn_err(h_open, ref_open) <= 1e-10, _turn_err(h_open, ref_open)
    # the walls change the answer
    assert _turn_err(h, ref_open) > 1e-6


def test_small_workload_three_turns_graph_equals_direct(gpu, orc):
    """Turns 2..n replay a captured graph; it must equal direct launches
    bit for bit, and the oracle within the FP64 bar."""
    _say("track small workload 3 turns graph vs direct")
    w = inputs.workload("small")
    ref = inputs.copy_parts(w["parts"])
    orc.track(ref, w["grid"], w["lattice"], 3)
    outs = []
    for use_graph in (True, False):
        with gpu.Context(w["grid"]) as ctx:
            ctx.set_option(gpu.OPT_USE_GRAPH, int(use_graph))
            d = _dev(w["parts"])
            ctx.track(d, w["lattice"], 3)
            outs.append(_host(d))
    for k in COORDS:
        np.testing.assert_array_equal(outs[0][k], outs[1][k])
    assert _turn_err(outs[0], ref) <= 1e-10


def test_turn_starting_and_ending_with_elements_and_lost_particles(gpu, orc):
    """A lattice with elements before the first and after the last SC
    location, several SC locations with different kappa, and a beam wide
    enough that particles leave the grid and are frozen."""
    _say("track irregular lattice with losses")
    g = inputs.make_grid(32, 32, 3e-3)
    p = inputs.gaussian_beam(20_000, 15)
    mx = inputs.rotation(0.41)
    my = inputs.rotation(0.57)
    lat = np.concatenate([inputs.lin2x2(mx, my), inputs.sext_thin(40.0), inputs.sc_kick(3e-8),
                          inputs.lin2x2(mx, my), inputs.lin2x2(my, mx), inputs.sc_kick(7e-8),
                          inputs.lin2x2(mx, mx), inputs.sc_kick(2e-8), inputs.lin2x2(my, my),
                          inputs.sext_thin(-25.0)])
    ref = inputs.copy_parts(p)
    orc.track(ref, g, lat, 4)
    with gpu.Context(g) as ctx:
        d = _dev(p)
        ctx.track(d, lat, 4)
        h = _host(d)
    assert 0 < int(ref["lost"].sum()) < 20_000
    np.testing.assert_array_equal(h["lost"], ref["lost"])
    assert _turn_err(h, ref) <= 1e-10


@pytest.fixture(scope="module")
def production_one_turn_reference(orc):
    w = inputs.workload("production")
    ref = inputs.copy_parts(w["parts"])
    orc.track(ref, w["grid"], w["lattice"], 1)
    return w, ref


def test_production_workload_one_turn_fp64(gpu, production_one_turn_reference):
    """Full production shape (1e6 particles, 128^2, 100 SC steps with 4x4
    maps and sextupoles), the launch configuration the benchmark times."""
    _say("track production workload 1 turn fp64 (1e6 particles)")
    w, ref = production_one_turn_reference
    with gpu.Context(w["grid"]) as ctx:
        d = _dev(w["parts"])
        ctx.track(d, w["lattice"], 1)
        h = _host(d)
    np.testing.assert_array_equal(h["lost"], ref["lost"])
    assert _turn_err(h, ref) <= 1e-10, _turn_err(h, ref)


def test_mixed_precision_small_workload(gpu, orc):
    """Mixed form vs FP64 oracle: one-turn coordinates and, over 50 turns,
    the rms emittance against the FP64 GPU form."""
    _say("track small workload mixed precision")
    from tests.physics import rms_emittance
    w = inputs.workload("small")
    ref = inputs.copy_parts(w["parts"])
    orc.track(ref, w["grid"], w["lattice"], 1)
    with gpu.Context(w["grid"], "mixed") as ctx:
        d = _dev(w["parts"])
        ctx.track(d, w["lattice"], 1)
        h = _host(d)
    # Bar derived from the FP32 field bar: each of the n_sc kicks of the turn
    # carries at most 1e-5 * max|E| * kappa of error, so the one-turn momentum
    # error is below n_sc * 1e-5 * kappa * max|E| (relative to the rms momenta).
    q, n_in = orc.deposit(inputs.copy_parts(w["parts"]), w["grid"])
    ex0, ey0 = orc.solve(q, 1.0 / ((1 << 24) * w["n"]), w["grid"])
    kappa = float(w["lattice"]["p"][w["lattice"]["kind"] == inputs.SC][0, 0])
    n_sc = int((w["lattice"]["kind"] == inputs.SC).sum())
    emax = max(np.abs(ex0).max(), np.abs(ey0).max())
    bar = 2 * n_sc * 1e-5 * kappa * emax / min(ref["px"].std(), ref["py"].std())
    err1 = _turn_err(h, ref)
    print(f"[mixed] one-turn coordinate error {err1:.3e} (bar {bar:.3e})", flush=True)
    assert err1 <= bar, (err1, bar)
    hs = []
    for prec in ("fp64", "mixed"):
        with gpu.Context(w["grid"], prec) as ctx:
            d = _dev(w["parts"])
            ctx.track(d, w["lattice"], 50)
            hs.append(_host(d))
    for u, pu in (("x", "px"), ("y", "py")):
        e64 = rms_emittance(hs[0][u], hs[0][pu], hs[0]["lost"] == 0)
        e32 = rms_emittance(hs[1][u], hs[1][pu], hs[1]["lost"] == 0)
        print(f"[mixed] emittance {u} after 50 turns: rel diff {abs(e32 / e64 - 1):.3e}",
              flush=True)
        assert abs(e32 / e64 - 1) <= 1e-4, (u, e32, e64)


@pytest.mark.parametrize("precision,bar", [("fp64", 1e-10), ("mixed", None)])
def test_long_bunch_weighted_kicks_on_256_grid(gpu, orc, precision, bar):
    """2.5D form on the large workload's geometry: KV 2:1 beam, per-particle
    line-density kick weights, 256^2 grid; 8 segments, 2 turns (a short ring
    so the oracle's direct-sum solve stays quick)."""
    _say(f"track long bunch 256^2 weighted kicks {precision}")
    w = inputs.workload("large", n=200_000)
    lat = inputs.ring(4.2, 4.3, 8, float(w["lattice"]["p"][w["lattice"]["kind"] == inputs.SC][0, 0]) * 25)
    ref = inputs.copy_parts(w["parts"])
    orc.track(ref, w["grid"], lat, 2)
    with gpu.Context(w["grid"], precision) as ctx:
        d = _dev(w["parts"])
        ctx.track(d, lat, 2)
        h = _host(d)
    np.testing.assert_array_equal(h["lost"], ref["lost"])
    err = _turn_err(h, ref)
    if bar is None:
        # FP32 field bar (1e-5 relative) over the 16 kicks, relative to rms momenta
        q, _ = orc.deposit(inputs.copy_parts(w["parts"]), w["grid"])
        ex0, ey0 = orc.solve(q, 1.0 / ((1 << 24) * w["n"]), w["grid"])
        kappa = float(lat["p"][lat["kind"] == inputs.SC][0, 0])
        emax = max(np.abs(ex0).max(), np.abs(ey0).max())
        bar = 2 * 16 * 1e-5 * kappa * emax / min(ref["px"].std(), ref["py"].std())
    print(f"[long bunch {precision}] two-turn coordinate error {err:.3e} (bar {bar:.3e})", flush=True)
    assert err <= bar, (err, bar)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_large_workload_full_size_one_step(gpu, orc, precision):
    """The large workload at full size (1e7 KV long-bunch particles with kick
    weights, 256^2 grid) in the default launch shape: deposit bit-exact, field
    within the precision's bar, and one step (map, deposit, solve, weighted
    kick) against the oracle."""
    import torch
    _say(f"large workload full size ({precision}): deposit and solve")
    w = inputs.workload("large")
    g = w["grid"]
    ref = inputs.copy_parts(w["parts"])
    q_ref, n_ref = orc.deposit(ref, g)
    scale = 1.0 / ((1 << 24) * w["n"])
    with gpu.Context(g, precision) as ctx:
        d = _dev(w["parts"])
        rho, n_in = ctx.deposit(d)
        np.testing.assert_array_equal(rho.cpu().numpy(), q_ref)
        assert int(n_in.item()) == n_ref
        ex, ey = ctx.solve(rho, scale)
        ex = ex.double().cpu().numpy()
        ey = ey.double().cpu().numpy()
    ex_ref, ey_ref = orc.solve(q_ref, scale, g)
    tol = 1e-12 if precision == "fp64" else 1e-5
    assert _field_err(ex, ex_ref) <= tol, _field_err(ex, ex_ref)
    assert _field_err(ey, ey_ref) <= tol, _field_err(ey, ey_ref)
    _say(f"large workload full size ({precision}): one step")
    lat = w["lattice"][:2]  # one segment: map, SC kick
    assert list(lat["kind"]) == [inputs.LIN2X2, inputs.SC]
    ref = inputs.copy_parts(w["parts"])
    orc.track(ref, g, lat, 1)
    with gpu.Context(g, precision) as ctx:
        d = _dev(w["parts"])
        ctx.track(d, lat, 1)
        h = _host(d)
    np.testing.assert_array_equal(h["lost"], ref["lost"])
    err = _turn_err(h, ref)
    if precision == "fp64":
        bar = 1e-10
    else:
        # one kick with the FP32 field bar, relative to the rms momenta
        kappa = float(lat["p"][1, 0])
        emax = max(np.abs(ex_ref).max(), np.abs(ey_ref).max())
        bar = 2 * 1e-5 * kappa * emax / min(ref["px"].std(), ref["py"].std())
    print(f"[large {precision}] one-step coordinate error {err:.3e} (bar {bar:.3e})", flush=True)
    assert err <= bar, (err, bar)



def test_large_workload_full_size_two_steps_streamed(gpu, orc):
    """Two segments of the large workload at full size in FP64: the second
    pass kicks and deposits with the first pass's boxes known, in the
    streamed form (the arrays exceed half the last-level cache) and with the
    charge tile's margin narrowed so the FP64 field box fits beside it.
    Coordinates against the oracle after both steps and the final kick."""
    _say("large workload full size (fp64): two steps, streamed fused pass")
    w = inputs.workload("large")
    g = w["grid"]
    lat = w["lattice"][:4]  # map, SC kick, map, SC kick
    assert list(lat["kind"]) == [inputs.LIN2X2, inputs.SC, inputs.LIN2X2, inputs.SC]
    ref = inputs.copy_parts(w["parts"])
    orc.track(ref, g, lat, 1)
    with gpu.Context(g, "fp64") as ctx:
        d = _dev(w["parts"])
        ctx.track(d, lat, 1)
        h = _host(d)
    np.testing.assert_array_equal(h["lost"], ref["lost"])
    err = _turn_err(h, ref)
    print(f"[large fp64 two steps] coordinate error {err:.3e}", flush=True)
    assert err <= 1e-10, err


def _moments(p):
    """Alive count, means and rms emittances written out from their
    definition (population moments about the mean, FP64) over the
    particles not lost."""
    m = p["lost"] == 0
    x, px, y, py = (np.asarray(p[k])[m] for k in ("x", "px", "y", "py"))

    def emit(a, b):
        da, db = a - a.mean(), b - b.mean()
        return np.sqrt((da * da).mean() * (db * db).mean() - (da * db).mean() ** 2)

    return int(m.sum()), [v.mean() for v in (x, px, y, py)], emit(x, px), emit(y, py), \
        [v.std() for v in (x, px, y, py)]


def _check_diag(got, p):
    n, means, ex, ey, stds = _moments(p)
    assert got["alive"] == n
    for g_, w_, s_ in zip(got["mean"], means, stds):
        assert abs(g_ - w_) <= 1e-12 * s_, (g_, w_)
    assert abs(got["emit_x"] / ex - 1.0) < 1e-11, (got["emit_x"], ex)
    assert abs(got["emit_y"] / ey - 1.0) < 1e-11, (got["emit_y"], ey)


def test_diagnostics_match_their_definition(gpu):
    """scpic_diagnose, and the diagnostics scpic_track returns after its last
    turn, against the moments written out in numpy: an off-centre beam with a
    tenth of its particles lost, then the same beam after two turns; the two
    calls on the same arrays agree exactly (fixed-order reductions)."""
    _say("beam diagnostics vs their definition")
    w = inputs.workload("small")
    parts = inputs.copy_parts(w["parts"])
    rng = np.random.Generator(np.random.PCG64(inputs.SEED_BASE + 77))
    parts["lost"][rng.random(parts["x"].shape[0]) < 0.1] = 1
    parts["x"] = parts["x"] + 0.3 * parts["x"].std()
    parts["py"] = parts["py"] - 0.2 * parts["py"].std()
    with gpu.Context(w["grid"]) as ctx:
        d = _dev(parts)
        _check_diag(ctx.diagnose(d), parts)
        tracked = ctx.track(d, w["lattice"], 2, diag=True)
        _check_diag(tracked, _host(d))
        assert ctx.diagnose(d) == tracked
        none = _dev(inputs.gaussian_beam(0, 1))
        assert ctx.diagnose(none) == {"alive": 0, "mean": [0.0] * 4, "emit_x": 0.0,
                                      "emit_y": 0.0}
        gone = inputs.gaussian_beam(500, 3)
        gone["lost"][:] = 1
        assert ctx.diagnose(_dev(gone))["alive"] == 0

def test_zero_particles_and_no_sc_lattice(gpu, orc):
    _say("track n=0 and lattice without SC")
    g = inputs.make_grid(32)
    with gpu.Context(g) as ctx:
        d = _dev(inputs.gaussian_beam(0, 1))
        ctx.track(d, inputs.workload("small")["lattice"], 2)
        p = inputs.gaussian_beam(5000, 16)
        ref = inputs.copy_parts(p)
        lat = inputs.ring(4.2, 4.3, 16, kappa=None)
        orc.track(ref, g, lat, 3)
        d = _dev(p)
        ctx.track(d, lat, 3)
        h = _host(d)
    for k in COORDS:
        np.testing.assert_array_equal(h[k], ref[k])
