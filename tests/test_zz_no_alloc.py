"""GPU check of lpc_pm_force_noalloc, the force entry point that takes no workspace and allocates nothing: its
output equals lpc_pm_force's bit for bit (same kernels, same integer deposit) on two calls in a row, the second with a
smaller input (the static scratch keeps the first call's contents, so anything left uncleared would show), and an
input too large for the static scratch is rejected before anything runs."""
import numpy as np
import pytest

import synth
from tests.gpu_util import requires_gpu, say, to_dev, to_np, torch

pytestmark = [pytest.mark.gpu, requires_gpu]


def both(lpc, pos, nm, box, p):
    n = pos.shape[1]
    geom = lpc.geometry(0, nm, box)
    step = lpc.stepping(deconv_power=p)
    pd = to_dev(pos)
    ws = lpc.workspace(geom, lpc.LPC_OP_PM_FORCE, n_particles=n)
    g_ref = torch.empty((3, n), dtype=torch.float32, device="cuda")
    d_ref = torch.empty((nm, nm, nm), dtype=torch.int64, device="cuda")
    lpc.lpc_pm_force(geom, step, pd, g_ref, ws, density_out=d_ref)
    g = torch.full((3, n), float("nan"), dtype=torch.float32, device="cuda")
    d = torch.full((nm, nm, nm), -1, dtype=torch.int64, device="cuda")
    lpc.lpc_pm_force_noalloc(geom, step, pd, g, density_out=d)
    g2 = torch.full((3, n), float("nan"), dtype=torch.float32, device="cuda")
    lpc.lpc_pm_force_noalloc(geom, step, pd, g2)  # without the density output: the FP32 contrast path
    return to_np(g_ref), to_np(d_ref), to_np(g), to_np(d), to_np(g2)


def test_noalloc_equals_workspace_entry_point():
    from paper_1506_03737_amd import lpc
    cases = [(synth.clustered_positions(21, 300001, 400.0), 96, 400.0, 1),   # first: the larger input
             (synth.uniform_positions(22, 5003, 100.0), 48, 100.0, 2)]       # second: smaller mesh and count
    for pos, nm, box, p in cases:
        say(f"noalloc: n={pos.shape[1]} nm={nm} p={p}")
        g_ref, d_ref, g, d, g2 = both(lpc, pos, nm, box, p)
        assert np.array_equal(d, d_ref)
        assert np.array_equal(g, g_ref)
        assert np.array_equal(g2, g_ref)


def test_noalloc_rejects_inputs_beyond_the_scratch():
    from paper_1506_03737_amd import lpc
    nm, n = 256, 1000
    geom = lpc.geometry(0, nm, 500.0)
    assert lpc.lpc_workspace_bytes(geom, lpc.LPC_OP_PM_FORCE, n) > lpc.NOALLOC_SCRATCH_BYTES
    say("noalloc: too large")
    pos = to_dev(synth.uniform_positions(23, n, 500.0))
    g = torch.empty((3, n), dtype=torch.float32, device="cuda")
    with pytest.raises(lpc.LpcError) as e:
        lpc.lpc_pm_force_noalloc(geom, lpc.stepping(), pos, g)
    assert e.value.status == -3
    assert "LPC_NOALLOC_SCRATCH_BYTES" in str(e.value)
