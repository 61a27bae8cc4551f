"""Batched tracking of independent beams (scpic_track_batched), through the C
ABI, against the FP64 CPU oracle and against the single-beam path.

Bars:
  batched vs single-beam GPU path   bit-exact (coordinates, lost flags, field):
                                    the same kernels' arithmetic on each beam
  one turn vs the oracle            max|u - u_ref| / rms(u_ref) <= 1e-10 (FP64)
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


def _beam(parts, offsets, k):
    a, b = int(offsets[k]), int(offsets[k + 1])
    return {key: v[a:b].copy() for key, v in parts.items()}


def _turn_err(h, ref):
    if ref["x"].shape[0] == 0:
        return 0.0
    return max(np.abs(h[k] - ref[k]).max() / max(ref[k].std(), 1e-300) for k in COORDS)


def _mixed_batch():
    """Six beams: different sizes (one empty, one below a workgroup), grids
    (square, anisotropic, rectangular, and 100 x 36 whose sides are not
    powers of two), tunes and element kinds, one shared schedule of 16 SC
    locations per turn."""
    eps = 1e-6
    kappa = inputs.kappa_for_tune_shift(-0.2, eps, 16)
    sizes = [3000, 0, 12001, 700, 20000, 9001]
    grids = [inputs.make_grid(32), inputs.make_grid(64), inputs.make_grid(64, 64, 5e-3, 7e-3),
             inputs.make_grid(16, 32, 6e-3, 6e-3), inputs.make_grid(64),
             inputs.make_grid(100, 36, 6e-3, 5e-3)]
    lattices = [inputs.ring(4.2, 4.3, 16, kappa),
                inputs.ring(4.1, 4.2, 16, kappa),
                inputs.ring(4.31, 4.17, 16, 2 * kappa, four_by_four=True, k2l=5.0, sext_every=4),
                inputs.ring(4.05, 4.08, 16, kappa),
                inputs.ring(4.45, 4.25, 16, kappa, four_by_four=True),
                inputs.ring(4.22, 4.33, 16, kappa)]
    beams = [inputs.gaussian_beam(n, 500 + k) for k, n in enumerate(sizes)]
    parts, offsets = inputs.concat_parts(beams)
    return parts, offsets, grids, lattices


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_equals_single_beam_path(gpu, precision):
    _say(f"batch of 6 beams, 3 turns, {precision}: batched == single-beam, bit-exact")
    parts, offsets, grids, lattices = _mixed_batch()
    with gpu.Batch(grids, offsets, precision) as b:
        d = _dev(parts)
        b.track(d, lattices, 3)
        got = _host(d)
        fields = [tuple(t.cpu().numpy() for t in b.get_field(k)) for k in range(len(grids))]
    for k in range(len(grids)):
        beam = _beam(parts, offsets, k)
        if beam["x"].shape[0] == 0:
            assert not np.any(fields[k][0]) and not np.any(fields[k][1])
            continue
        with gpu.Context(grids[k], precision) as ctx:
            dk = _dev(beam)
            ctx.track(dk, lattices[k], 3)
            want = _host(dk)
            ex, ey = (t.cpu().numpy() for t in ctx.get_field())
        mine = _beam(got, offsets, k)
        for key in COORDS + ("lost",):
            np.testing.assert_array_equal(mine[key], want[key], err_msg=f"beam {k} {key}")
        np.testing.assert_array_equal(fields[k][0], ex, err_msg=f"beam {k} ex")
        np.testing.assert_array_equal(fields[k][1], ey, err_msg=f"beam {k} ey")


def test_batch_with_a_wide_grid_equals_single_beam_path(gpu):
    """A batch whose widest grid has ny > 128 (a 64 x 256 grid beside a 64^2
    one) runs its row kernel on wider workgroups than a batch of grids up to
    128 wide; both beams still equal their single-beam runs bit for bit."""
    _say("batch with a 64x256 grid, 2 turns fp64: batched == single-beam, bit-exact")
    kappa = inputs.kappa_for_tune_shift(-0.2, 1e-6, 16)
    grids = [inputs.make_grid(64), inputs.make_grid(64, 256, 6e-3, 6e-3)]
    lattices = [inputs.ring(4.2, 4.3, 16, kappa), inputs.ring(4.12, 4.27, 16, kappa)]
    beams = [inputs.gaussian_beam(n, 700 + k) for k, n in enumerate((6000, 9000))]
    parts, offsets = inputs.concat_parts(beams)
    with gpu.Batch(grids, offsets) as b:
        d = _dev(parts)
        b.track(d, lattices, 2)
        got = _host(d)
        fields = [tuple(t.cpu().numpy() for t in b.get_field(k)) for k in range(len(grids))]
    for k in range(len(grids)):
        with gpu.Context(grids[k]) as ctx:
            dk = _dev(_beam(parts, offsets, k))
            ctx.track(dk, lattices[k], 2)
            want = _host(dk)
            ex, ey = (t.cpu().numpy() for t in ctx.get_field())
        mine = _beam(got, offsets, k)
        for key in COORDS + ("lost",):
            np.testing.assert_array_equal(mine[key], want[key], err_msg=f"beam {k} {key}")
        np.testing.assert_array_equal(fields[k][0], ex, err_msg=f"beam {k} ex")
        np.testing.assert_array_equal(fields[k][1], ey, err_msg=f"beam {k} ey")


def test_batch_one_turn_matches_oracle(gpu, orc):
    _say("batch of 6 beams, 1 turn fp64 vs oracle")
    parts, offsets, grids, lattices = _mixed_batch()
    with gpu.Batch(grids, offsets) as b:
        d = _dev(parts)
        b.track(d, lattices, 1)
        got = _host(d)
    for k in range(len(grids)):
        ref = _beam(parts, offsets, k)
        if ref["x"].shape[0] == 0:
            continue
        orc.track(ref, grids[k], lattices[k], 1)
        mine = _beam(got, offsets, k)
        np.testing.assert_array_equal(mine["lost"], ref["lost"], err_msg=f"beam {k}")
        assert _turn_err(mine, ref) <= 1e-10, (k, _turn_err(mine, ref))


def test_batch_rejects_rings_with_other_schedules(gpu):
    _say("batch schedule mismatch and size checks")
    parts, offsets, grids, lattices = _mixed_batch()
    kappa = inputs.kappa_for_tune_shift(-0.2, 1e-6, 8)
    bad = list(lattices)
    bad[2] = inputs.ring(4.2, 4.3, 8, kappa)  # 8 SC locations instead of 16
    with gpu.Batch(grids, offsets) as b:
        d = _dev(parts)
        with pytest.raises(gpu.ScpicError) as e:
            b.track(d, bad, 1)
        assert e.value.code == gpu.EUNSUPPORTED
        short = {k: v[:-1].contiguous() for k, v in d.items()}
        with pytest.raises(gpu.ScpicError) as e:
            b.track(short, lattices, 1)
        assert e.value.code == gpu.EINVAL
        # nothing was run: the particles are untouched
        np.testing.assert_array_equal(_host(d)["x"], parts["x"])


def test_tune_scan_batch_full_size(gpu, orc):
    """The 64-beam tune scan (8.1e6 particles, 64^2 and 128^2 grids): one turn
    of every beam against the oracle; then 200 turns, with four beams (the two
    smallest, the largest and the smallest of the lowest-tune row, which loses
    particles) equal bit for bit to their single-beam runs."""
    _say("tune scan batch: 64 beams, 8.1e6 particles")
    w = inputs.batch_workload()
    offsets, grids, lattices = w["offsets"], w["grids"], w["lattices"]
    with gpu.Batch(grids, offsets) as b:
        d = _dev(w["parts"])
        b.track(d, lattices, 1)
        one = _host(d)
        _say("tune scan batch: oracle, one turn of each beam")
        worst = 0.0
        for k in range(len(grids)):
            ref = _beam(w["parts"], offsets, k)
            orc.track(ref, grids[k], lattices[k], 1)
            mine = _beam(one, offsets, k)
            np.testing.assert_array_equal(mine["lost"], ref["lost"], err_msg=f"beam {k}")
            worst = max(worst, _turn_err(mine, ref))
        print(f"[batch] one turn, worst beam error {worst:.3e} of rms", flush=True)
        assert worst <= 1e-10
        _say("tune scan batch: 199 more turns")
        b.track(d, lattices, w["turns"] - 1)
        full = _host(d)
    sizes = w["sizes"]
    low_row = [k for k in range(len(grids)) if w["tunes"][k][1] == w["tunes"][0][1]]
    pick = sorted(set(list(np.argsort(sizes)[:2]) + [int(np.argmax(sizes))] +
                      [min(low_row, key=lambda k: sizes[k])]))
    lost_total = 0
    for k in pick:
        _say(f"tune scan batch: beam {k} (N={sizes[k]}) single-beam, {w['turns']} turns")
        beam = _beam(w["parts"], offsets, k)
        with gpu.Context(grids[k]) as ctx:
            dk = _dev(beam)
            ctx.track(dk, lattices[k], w["turns"])
            want = _host(dk)
        mine = _beam(full, offsets, k)
        for key in COORDS + ("lost",):
            np.testing.assert_array_equal(mine[key], want[key], err_msg=f"beam {k} {key}")
        lost_total += int(want["lost"].sum())
    alive = full["lost"] == 0
    assert all(np.isfinite(full[c][alive]).all() for c in COORDS)
    print(f"[batch] lost in the checked beams after {w['turns']} turns: {lost_total}",
          flush=True)


def test_autotune_picks_a_shape_and_keeps_results(gpu):
    _say("batch autotune on 5 beams, then 3 turns == single-beam path")
    parts, offsets, grids, lattices = _mixed_batch()
    with gpu.Batch(grids, offsets) as b:
        d = _dev(parts)
        threads, per_cu = b.autotune(d, lattices, trial_turns=1)
        print(f"[batch] autotune chose {threads} threads, {per_cu} workgroups per CU", flush=True)
        assert threads in (256, 512, 1024) and per_cu in (1, 2, 4)
        np.testing.assert_array_equal(_host(d)["x"], parts["x"])  # tuning ran on a copy
        b.track(d, lattices, 3)
        got = _host(d)
    for k in (0, 2, 4):
        beam = _beam(parts, offsets, k)
        with gpu.Context(grids[k]) as ctx:
            dk = _dev(beam)
            ctx.track(dk, lattices[k], 3)
            want = _host(dk)
        mine = _beam(got, offsets, k)
        for key in COORDS + ("lost",):
            np.testing.assert_array_equal(mine[key], want[key], err_msg=f"beam {k} {key}")
