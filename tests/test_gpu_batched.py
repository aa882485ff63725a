"""GPU parity of the batched run (lpc_cola_step_batched): several boxes of unequal mesh size, box side and particle
count advanced by one launch per stage.

Bar: bit-for-bit equality with separate lpc_cola_step calls on each box (the batched launches perform the same
per-element arithmetic and the same integer deposit), on the first call (graph recorded), on a replay of the
recorded graph, and with graphs switched off; and for one box, positions within 1e-5 L of the FP64 oracle.
"""
import functools

import numpy as np
import pytest

import synth
from oracle import cola as ocola
from oracle import ic as oic
from tests.gpu_util import particle_set, periodic_diff, requires_gpu, say, to_np, torch

pytestmark = [pytest.mark.gpu, requires_gpu]

C = synth.COSMOLOGY

# (n_side, n_mesh, box, seed): ragged mesh sizes (40 = 8 x 5, 48 = 16 x 3, 96; 36, whose last 16 x 8 x 32-cell sort
# tile is narrow along every axis) and unequal particle counts
BOXES = [(16, 32, 128.0, 11), (20, 40, 160.0, 12), (24, 48, 200.0, 13), (32, 96, 256.0, 14), (16, 48, 100.0, 15),
         (18, 36, 120.0, 16)]


def box_ic(n_side, box, seed):
    init = oic.initial_conditions(seed, n_side, box, synth.A_LIST[0], **C)
    return {k: init[k].astype(np.float32) for k in ("pos", "vel", "psi1", "psi2")}


def make_sets(lpc, ics):
    return [particle_set(lpc, ic["pos"], ic["vel"], ic["psi1"], ic["psi2"]) for ic in ics]


def single_runs(lpc, ics, boxes, a_list, step):
    out = []
    for ic, (n_side, nm, box, _) in zip(ics, boxes):
        ps = particle_set(lpc, ic["pos"], ic["vel"], ic["psi1"], ic["psi2"])
        geom = lpc.geometry(n_side, nm, box)
        ws = lpc.workspace(geom, lpc.LPC_OP_COLA_STEP)
        lpc.lpc_cola_step(geom, lpc.cosmology(**C), step, a_list, ps, ws)
        out.append((to_np(ps.pos), to_np(ps.vel)))
    return out


def batched_run(lpc, ics, boxes, a_list, step, ws=None):
    sets = make_sets(lpc, ics)
    entries = [(lpc.geometry(n, nm, L), ps) for ps, (n, nm, L, _) in zip(sets, boxes)]
    if ws is None:
        ws = lpc.workspace_batched(entries)
    lpc.lpc_cola_step_batched(entries, lpc.cosmology(**C), step, a_list, ws)
    return [(to_np(ps.pos), to_np(ps.vel)) for ps in sets], sets, entries, ws


@pytest.mark.parametrize("step_kw", [dict(), dict(cola=0, modified=0)], ids=["cola-modified", "pm-standard"])
def test_batched_equals_single_bitwise(step_kw):
    from paper_1506_03737_amd import lpc
    say(f"batched: {len(BOXES)} ragged boxes, {step_kw}")
    step = lpc.stepping(**step_kw)
    a = synth.A_LIST[:6]
    ics = [box_ic(n, L, seed) for (n, nm, L, seed) in BOXES]
    ref = single_runs(lpc, ics, BOXES, a, step)
    got, _, _, _ = batched_run(lpc, ics, BOXES, a, step)
    for i, ((x, v), (xr, vr)) in enumerate(zip(got, ref)):
        assert np.array_equal(x, xr), f"box {i}: positions differ"
        assert np.array_equal(v, vr), f"box {i}: velocities differ"


def test_graph_replay_and_direct_launch_agree():
    from paper_1506_03737_amd import lpc
    say("batched: graph record, replay, direct")
    step = lpc.stepping()
    a = synth.A_LIST[:4]
    ics = [box_ic(n, L, seed) for (n, nm, L, seed) in BOXES]
    first, sets, entries, ws = batched_run(lpc, ics, BOXES, a, step)
    # replay: same entries, same workspace, inputs reset in place
    for ps, ic in zip(sets, ics):
        for k in ("pos", "vel", "psi1", "psi2"):
            getattr(ps, k).copy_(torch.from_numpy(ic[k]))
    for rep in range(3):
        if rep > 0:
            for ps, ic in zip(sets, ics):
                for k in ("pos", "vel"):
                    getattr(ps, k).copy_(torch.from_numpy(ic[k]))
            torch.cuda.synchronize()
        lpc.lpc_cola_step_batched(entries, lpc.cosmology(**C), step, a, ws)
        torch.cuda.synchronize()
        for i, ps in enumerate(sets):
            assert np.array_equal(to_np(ps.pos), first[i][0]), f"replay {rep} box {i}"
            assert np.array_equal(to_np(ps.vel), first[i][1]), f"replay {rep} box {i}"
    lpc.lpc_graph_enable(False)
    try:
        direct, _, _, _ = batched_run(lpc, ics, BOXES, a, step)
    finally:
        lpc.lpc_graph_enable(True)
    for i in range(len(BOXES)):
        assert np.array_equal(direct[i][0], first[i][0])


def test_batched_box_matches_oracle():
    from paper_1506_03737_amd import lpc
    say("batched: box 3 against the oracle")
    step = lpc.stepping()
    a = synth.A_LIST
    boxes = BOXES[2:4]
    ics = [box_ic(n, L, seed) for (n, nm, L, seed) in boxes]
    got, _, _, _ = batched_run(lpc, ics, boxes, a, step)
    n, nm, L, _ = boxes[1]
    ic = ics[1]
    xr, vr = ocola.cola_run(ic["pos"], ic["vel"], ic["psi1"], ic["psi2"], a, C["omega_m"], nm, L)
    assert np.abs(periodic_diff(got[1][0], xr, L)).max() / L < 1e-5


def test_batch_of_one_and_errors():
    from paper_1506_03737_amd import lpc
    say("batched: one entry; argument errors")
    step = lpc.stepping()
    a = synth.A_LIST[:3]
    box = [BOXES[0]]
    ics = [box_ic(n, L, seed) for (n, nm, L, seed) in box]
    ref = single_runs(lpc, ics, box, a, step)
    got, sets, entries, ws = batched_run(lpc, ics, box, a, step)
    assert np.array_equal(got[0][0], ref[0][0])
    small = ws[: ws.numel() - 256]
    with pytest.raises(lpc.LpcError) as e:
        lpc.lpc_cola_step_batched(entries, lpc.cosmology(**C), step, a, small)
    assert e.value.status == -3
    bad = [(lpc.geometry(16, 14, 128.0), sets[0])]
    with pytest.raises(lpc.LpcError) as e:
        lpc.lpc_cola_step_batched(bad, lpc.cosmology(**C), step, a, ws)
    assert e.value.status == -2


@functools.lru_cache(maxsize=None)
def oracle_run(n_side, nm, box, seed):
    """The FP64 oracle's ten-step modified-COLA run of one box (cached across the tests that use it)."""
    ic = box_ic(n_side, box, seed)
    return ocola.cola_run(ic["pos"], ic["vel"], ic["psi1"], ic["psi2"], synth.A_LIST, C["omega_m"], nm, box)


@pytest.mark.parametrize("poisson_cols", [None, 8], ids=["builtin-widths", "poisson-8-chained"])
def test_batched_workload_shapes(poisson_cols):
    """One box of each shape of the 48-box workload (N = 96, 128, 160 with Nm = 2N, boxes 300, 450, 600 Mpc/h), so
    the batched launches take the 192, 256 and 320 meshes (compile-time FFT plans 8 8 3, 8 8 4, 8 8 5 and their half
    lengths) together, with the tile widths and points per thread shared across the three: every box equals its own
    lpc_cola_step run bit for bit over ten steps, and the N = 96 box is within 1e-5 L of the FP64 oracle. With the
    built-in widths the fused x pass takes 16-column tiles (its unchained form); with 8-column tiles, the width the
    autotuner picks at these meshes, it chains its three transforms through registers."""
    from paper_1506_03737_amd import lpc
    boxes = [(96, 192, 300.0, 1000), (128, 256, 450.0, 1001), (160, 320, 600.0, 1002)]
    say(f"batched: workload shapes 96/192, 128/256, 160/320, ten steps, poisson_cols={poisson_cols}")
    step = lpc.stepping()
    a = synth.A_LIST
    ics = [box_ic(n, L, seed) for (n, nm, L, seed) in boxes]
    try:
        if poisson_cols is not None:
            for _, nm, _, _ in boxes:
                lpc.lpc_fft_tiling_set(nm, dict(lpc.lpc_fft_tiling_default(nm), poisson_cols=poisson_cols))
        ref = single_runs(lpc, ics, boxes, a, step)
        got, _, _, _ = batched_run(lpc, ics, boxes, a, step)
    finally:
        lpc.lpc_fft_tiling_reset()
    for i, ((x, v), (xr, vr)) in enumerate(zip(got, ref)):
        assert np.array_equal(x, xr), f"box {i}: positions differ"
        assert np.array_equal(v, vr), f"box {i}: velocities differ"
    n, nm, L, seed = boxes[0]
    xr, vr = oracle_run(n, nm, L, seed)
    dx = np.abs(periodic_diff(got[0][0], xr, L)).max() / L
    dv = np.sqrt(np.mean((got[0][1] - vr) ** 2)) / np.sqrt(np.mean(vr**2))
    say(f"  N=96 box vs oracle: max |dx|/L = {dx:.3e}, rms |dv|/rms v = {dv:.3e}")
    assert dx < 1e-5
    assert dv < 1e-4


def test_two_768_boxes_equal_their_single_runs():
    """Two boxes of the single-box mesh (768^3, 128^3 particles each, 1000 and 700 Mpc/h) in one batched launch:
    each equals its own single run bit for bit over two steps (the batched jobs take the same kernel instances,
    including the fused x pass chained through registers, as one box alone)."""
    from paper_1506_03737_amd import lpc
    boxes = [(128, 768, 1000.0, 2001), (128, 768, 700.0, 2002)]
    say("batched: two 768^3 boxes against their single runs")
    step = lpc.stepping()
    a = synth.A_LIST[:3]
    ics = [box_ic(n, L, seed) for (n, nm, L, seed) in boxes]
    ref = single_runs(lpc, ics, boxes, a, step)
    got, _, _, _ = batched_run(lpc, ics, boxes, a, step)
    for i, ((x, v), (xr, vr)) in enumerate(zip(got, ref)):
        assert np.array_equal(x, xr), f"box {i}: positions differ"
        assert np.array_equal(v, vr), f"box {i}: velocities differ"
