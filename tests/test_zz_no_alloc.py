"""The allocation-free deposit (scpic_deposit_static) against the context's
deposit (scpic_deposit) and the FP64 CPU oracle: bit-exact charge grids, lost
flags and counts, over consecutive calls that share the static scratch (a
large call, then a smaller one on a smaller grid; the carry grid's overflow
path, then a plain call), and replays of a captured graph of the call."""
import sys

import numpy as np
import pytest

from paper_2010_11540_amd import inputs

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"\n[case] {msg}", flush=True)
    sys.stdout.flush()


def _static(gpu, g, d):
    import torch
    rho = torch.empty(g["nx"] * g["ny"], dtype=torch.int64, device="cuda")
    n_in = torch.empty(1, dtype=torch.int64, device="cuda")
    gpu.deposit_static(g, d, rho, n_in)
    torch.cuda.synchronize()
    return rho.cpu().numpy(), int(n_in.item())


def _context(gpu, g, d):
    import torch
    with gpu.Context(g) as ctx:
        rho, n_in = ctx.deposit(d)
        torch.cuda.synchronize()
        return rho.cpu().numpy(), int(n_in.item())


def test_static_deposit_matches_context_deposit_on_two_calls(gpu, orc):
    from paper_2010_11540_amd.scpic import to_device
    cases = [(1_000_003, 128, 128, 31), (10_001, 64, 64, 32)]  # the second is smaller
    for n, nx, ny, seed in cases:
        _say(f"static deposit n={n} grid={nx}x{ny} seed={seed}")
        g = inputs.make_grid(nx, ny, 4.5e-3, 5e-3)
        p = inputs.gaussian_beam(n, seed)
        ref = inputs.copy_parts(p)
        q_ref, n_ref = orc.deposit(ref, g)
        d_static, d_ctx = to_device(p), to_device(p)
        q_s, n_s = _static(gpu, g, d_static)
        q_c, n_c = _context(gpu, g, d_ctx)
        np.testing.assert_array_equal(q_s, q_c)
        np.testing.assert_array_equal(q_s, q_ref)
        assert n_s == n_c == n_ref
        np.testing.assert_array_equal(d_static["lost"].cpu().numpy(), d_ctx["lost"].cpu().numpy())
        np.testing.assert_array_equal(d_static["lost"].cpu().numpy(), ref["lost"])


def test_static_deposit_overflow_then_plain_call(gpu, orc):
    """2^18 particles on one node wrap the 32-bit LDS cells into the carry
    grid; the next, smaller call must start from a cleared carry grid."""
    from paper_2010_11540_amd.scpic import to_device
    g = inputs.make_grid(64, 64, 4.5e-3, 5e-3)
    n = 1 << 18
    p = {"x": np.full(n, g["x_min"] + 20 * g["dx"]), "px": np.zeros(n),
         "y": np.full(n, g["y_min"] + 30 * g["dy"]), "py": np.zeros(n),
         "lost": np.zeros(n, dtype=np.uint8)}
    _say("static deposit overflow path: 2^18 particles on one node, 64x64")
    q_ref, n_ref = orc.deposit(inputs.copy_parts(p), g)
    q_s, n_s = _static(gpu, g, to_device(p))
    np.testing.assert_array_equal(q_s, q_ref)
    assert n_s == n_ref == n
    g2 = inputs.make_grid(32, 32, 4.5e-3, 5e-3)
    p2 = inputs.gaussian_beam(5_003, 33)
    _say("static deposit after the overflow: n=5003 grid=32x32")
    q2_ref, n2_ref = orc.deposit(inputs.copy_parts(p2), g2)
    q2_s, n2_s = _static(gpu, g2, to_device(p2))
    np.testing.assert_array_equal(q2_s, q2_ref)
    assert n2_s == n2_ref


def test_static_deposit_replays_of_a_captured_graph(gpu, orc):
    """Captured once, replayed three times with eager work and
    synchronisations between the replays: every replay equals the eager
    call's result."""
    import torch
    from paper_2010_11540_amd.scpic import to_device
    g = inputs.make_grid(128, 128, 4.5e-3, 5e-3)
    p = inputs.gaussian_beam(300_007, 34)
    _say("static deposit captured in a graph: n=300007 grid=128x128")
    d = to_device(p)
    q_eager, n_eager = _static(gpu, g, d)  # uncaptured first call on the device
    rho = torch.empty(128 * 128, dtype=torch.int64, device="cuda")
    n_in = torch.empty(1, dtype=torch.int64, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side):
        gpu.deposit_static(g, d, rho, n_in, stream=side)
    torch.cuda.synchronize()
    other = inputs.gaussian_beam(20_011, 35)
    for r in range(3):
        rho.fill_(-7)
        n_in.fill_(-7)
        graph.replay()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(rho.cpu().numpy(), q_eager)
        assert int(n_in.item()) == n_eager
        # eager work on the same scratch between the replays
        g_o = inputs.make_grid(64, 64, 4.5e-3, 5e-3)
        q_o, _ = _static(gpu, g_o, to_device(other))
        np.testing.assert_array_equal(q_o, orc.deposit(inputs.copy_parts(other), g_o)[0])
