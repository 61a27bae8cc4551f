"""The long-bunch line density on the HIP path (Sec. IV: per-step histogram
of sigma, transverse kick scaled by lambda/lambda_peak, longitudinal kick from
the grounded-pipe potential), through the C ABI, against the FP64 oracle.

Bars:
  line tables lw, ld            bit-exact (integer histogram, same divisions)
  node potential (nodes -1..n)  max|phi - phi_ref| / max|phi_ref| <= 1e-12 (FP64)
  one step / one turn           max|u - u_ref| / rms(u_ref) <= 1e-10 per
                                coordinate, p_sigma included (FP64)
  mixed form, one turn          the FP32 field bar over the turn's kicks for the
                                transverse momenta; for p_sigma the FP32 bar on
                                phi times gamma0 kappa max|ld| per kick
"""
import sys

import numpy as np
import pytest

from paper_2010_11540_amd import inputs

pytestmark = pytest.mark.gpu

COORDS6 = ("x", "px", "y", "py", "sigma", "psigma")


def _say(msg):
    print(f"\n[case] {msg}", flush=True)
    sys.stdout.flush()


def _dev(parts):
    from paper_2010_11540_amd.scpic import to_device
    return to_device(parts)


def _host(parts):
    return {k: v.cpu().numpy() for k, v in parts.items()}


def _err6(h, ref):
    return max(np.abs(h[k] - ref[k]).max() / max(ref[k].std(), 1e-300) for k in COORDS6)


def _ctx(gpu, grid, line, precision="fp64"):
    ctx = gpu.Context(grid, precision)
    ctx.set_option(gpu.OPT_SOLVER, gpu.SOLVER_PIPE)
    ctx.set_line_density(line)
    return ctx


def _beam(n, seed):
    bx, by = inputs.fodo_beta(16, 4.2)
    return inputs.gaussian_beam6d(n, seed, 1e-3, 1e-3 / bx, 1e-3 * (by / bx) ** 0.5,
                                  1e-3 / (bx * by) ** 0.5)


@pytest.mark.parametrize("n,nx,nz", [(20_000, 64, 128), (3_001, 32, 64), (150_000, 128, 128)])
def test_line_step_matches_oracle(gpu, orc, n, nx, nz):
    """One space-charge step (deposit with the line histogram, pipe solve,
    line-weighted transverse kick and longitudinal kick) as a one-element
    turn; tables bit-exact, potential and coordinates within the bars."""
    _say(f"line step n={n} grid {nx}^2 nz={nz}")
    grid = inputs.make_grid(nx)
    line = inputs.make_line(4.0, nz)
    p0 = _beam(n, 70 + n)
    p0["sigma"][:2] = (9.0, -9.0)  # outside the line: lost at the deposit
    kappa = 3e-7
    ref = inputs.copy_parts(p0)
    lw, ld, phi, _ = orc.space_charge_line(ref, grid, line, 1.0 / ((1 << 24) * n), kappa)
    with _ctx(gpu, grid, line) as ctx:
        d = _dev(p0)
        ctx.track(d, inputs.sc_kick(kappa), 1)
        h = _host(d)
        glw, gld = (t.cpu().numpy() for t in ctx.get_line_state())
        gphi = ctx.get_potential().cpu().numpy()
    np.testing.assert_array_equal(h["lost"], ref["lost"])
    assert ref["lost"].sum() > 0
    np.testing.assert_array_equal(glw, lw)
    np.testing.assert_array_equal(gld, ld)
    perr = np.abs(gphi - phi).max() / np.abs(phi).max()  # nodes -1..n, walls included
    err = _err6(h, ref)
    print(f"[line step] phi error {perr:.3e}, coordinate error {err:.3e} of rms", flush=True)
    assert perr <= 1e-12
    assert err <= 1e-10
    assert np.any(h["psigma"] != p0["psigma"])


@pytest.mark.parametrize("use_graph", [True, False])
def test_line_small_one_turn_fp64(gpu, orc, use_graph):
    _say(f"line_small workload 1 turn fp64 (graph={use_graph})")
    w = inputs.workload("line_small")
    ref = inputs.copy_parts(w["parts"])
    orc.track_line(ref, w["grid"], w["line"], w["lattice"], 1)
    with _ctx(gpu, w["grid"], w["line"]) as ctx:
        ctx.set_option(gpu.OPT_USE_GRAPH, int(use_graph))
        d = _dev(w["parts"])
        ctx.track(d, w["lattice"], 1)
        h = _host(d)
    np.testing.assert_array_equal(h["lost"], ref["lost"])
    err = _err6(h, ref)
    print(f"[line small] one-turn error {err:.3e} of rms", flush=True)
    assert err <= 1e-10, err


def test_line_small_one_turn_mixed(gpu, orc):
    _say("line_small workload 1 turn mixed")
    w = inputs.workload("line_small")
    ref = inputs.copy_parts(w["parts"])
    orc.track_line(ref, w["grid"], w["line"], w["lattice"], 1)
    with _ctx(gpu, w["grid"], w["line"], "mixed") as ctx:
        d = _dev(w["parts"])
        ctx.track(d, w["lattice"], 1)
        h = _host(d)
    np.testing.assert_array_equal(h["lost"], ref["lost"])
    lat = w["lattice"]
    kappa = float(lat["p"][lat["kind"] == inputs.SC][0, 0])
    n_sc = int((lat["kind"] == inputs.SC).sum())
    probe = inputs.copy_parts(w["parts"])
    _, ld, phi, _ = orc.space_charge_line(probe, w["grid"], w["line"],
                                          1.0 / ((1 << 24) * w["n"]), kappa)
    q, _ = orc.deposit(inputs.copy_parts(w["parts"]), w["grid"])
    ex0, ey0 = orc.solve(q, 1.0 / ((1 << 24) * w["n"]), w["grid"], solver="pipe")
    emax = max(np.abs(ex0).max(), np.abs(ey0).max())
    bar_t = 2 * n_sc * 1e-5 * kappa * emax / min(ref["px"].std(), ref["py"].std())
    bar_l = (2 * n_sc * 1e-5 * w["line"]["gamma0"] * kappa * np.abs(phi).max() *
             np.abs(ld).max() / ref["psigma"].std())
    et = max(np.abs(h[k] - ref[k]).max() / ref[k].std() for k in ("x", "px", "y", "py"))
    el = np.abs(h["psigma"] - ref["psigma"]).max() / ref["psigma"].std()
    print(f"[line small mixed] transverse {et:.3e} (bar {bar_t:.3e}), p_sigma {el:.3e} "
          f"(bar {bar_l:.3e})", flush=True)
    assert et <= bar_t and el <= bar_l


@pytest.fixture(scope="module")
def line_one_turn_reference(orc):
    w = inputs.workload("line")
    ref = inputs.copy_parts(w["parts"])
    orc.track_line(ref, w["grid"], w["line"], w["lattice"], 1)
    return w, ref


def test_line_workload_full_size_one_turn_fp64(gpu, line_one_turn_reference):
    """The long-bunch workload at full size (1e6 particles, 128^2 pipe, 128
    line nodes, 100 thick FODO cells) in the launch configuration the
    benchmark times."""
    _say("line workload full size 1 turn fp64 (1e6 particles)")
    w, ref = line_one_turn_reference
    with _ctx(gpu, w["grid"], w["line"]) as ctx:
        d = _dev(w["parts"])
        ctx.track(d, w["lattice"], 1)
        h = _host(d)
    np.testing.assert_array_equal(h["lost"], ref["lost"])
    err = _err6(h, ref)
    print(f"[line full] one-turn error {err:.3e} of rms", flush=True)
    assert err <= 1e-10, err


def test_line_density_argument_checks(gpu):
    _say("line density argument checks")
    w = inputs.workload("line_small")
    lat = w["lattice"]
    with gpu.Context(w["grid"]) as ctx:
        d = _dev(w["parts"])
        with pytest.raises(gpu.ScpicError) as e:
            ctx.get_line_state()
        assert e.value.code == gpu.EINVAL
        for bad in ({"nz": 4, "z_min": -1.0, "dz": 0.1, "gamma0": 4.0},
                    {"nz": 1024, "z_min": -1.0, "dz": 0.1, "gamma0": 4.0},
                    {"nz": 64, "z_min": -1.0, "dz": 0.0, "gamma0": 4.0},
                    {"nz": 64, "z_min": -1.0, "dz": 0.1, "gamma0": 0.5}):
            with pytest.raises(gpu.ScpicError) as e:
                ctx.set_line_density(bad)
            assert e.value.code == gpu.EINVAL
        ctx.set_line_density(w["line"])
        with pytest.raises(gpu.ScpicError) as e:  # open boundary: no absolute potential
            ctx.track(d, lat, 1)
        assert e.value.code == gpu.EUNSUPPORTED
        ctx.set_option(gpu.OPT_SOLVER, gpu.SOLVER_PIPE)
        four = {k: v for k, v in d.items() if k not in ("sigma", "psigma")}
        with pytest.raises(gpu.ScpicError) as e:
            ctx.track(four, inputs.ring(4.2, 4.3, 4, 1e-9), 1)
        assert e.value.code == gpu.EINVAL
        import torch
        weighted = dict(d, w=torch.ones_like(d["x"], dtype=torch.float32))
        with pytest.raises(gpu.ScpicError) as e:
            ctx.track(weighted, lat, 1)
        assert e.value.code == gpu.EINVAL
        h = _host(d)
    for k in COORDS6:
        np.testing.assert_array_equal(h[k], w["parts"][k])


def test_line_density_off_again_is_plain_pipe_tracking(gpu):
    _say("line density on then off == never on")
    w = inputs.workload("line_small")
    outs = []
    for toggle in (False, True):
        with gpu.Context(w["grid"]) as ctx:
            ctx.set_option(gpu.OPT_SOLVER, gpu.SOLVER_PIPE)
            if toggle:
                ctx.set_line_density(w["line"])
                ctx.set_line_density(None)
            d = _dev(w["parts"])
            ctx.track(d, w["lattice"], 2)
            outs.append(_host(d))
    for k in COORDS6 + ("lost",):
        np.testing.assert_array_equal(outs[0][k], outs[1][k])
    np.testing.assert_array_equal(outs[0]["psigma"], w["parts"]["psigma"])


def test_per_element_calls_stay_transverse_with_the_line_on(gpu, orc):
    """scpic_deposit and scpic_kick ignore the line density: the deposit of
    four-dimensional particles is the oracle's, and a kick with a given field
    equals the same kick on a context without the line."""
    _say("per-element deposit and kick with the line density on")
    w = inputs.workload("line_small")
    four = {k: v for k, v in w["parts"].items() if k not in ("sigma", "psigma")}
    q_ref, n_ref = orc.deposit(inputs.copy_parts(four), w["grid"])
    ex, ey = orc.solve(q_ref, 1.0 / ((1 << 24) * w["n"]), w["grid"], solver="pipe")
    import torch
    outs = []
    for line_on in (True, False):
        with gpu.Context(w["grid"]) as ctx:
            ctx.set_option(gpu.OPT_SOLVER, gpu.SOLVER_PIPE)
            if line_on:
                ctx.set_line_density(w["line"])
            d = _dev(four)
            rho, n_in = ctx.deposit(d)
            np.testing.assert_array_equal(rho.cpu().numpy(), q_ref)
            assert int(n_in.item()) == n_ref
            d6 = _dev(w["parts"])
            ctx.kick(d6, torch.from_numpy(ex).cuda(), torch.from_numpy(ey).cuda(), 3e-7)
            outs.append(_host(d6))
    for k in COORDS6 + ("lost",):
        np.testing.assert_array_equal(outs[0][k], outs[1][k])
