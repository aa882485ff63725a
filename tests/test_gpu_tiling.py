"""FFT tile widths (lpc_fft_tiling_*) and their autotuner on the GPU.

A tile width only decides how many independent 1-D transforms share one LDS tile; the arithmetic of each transform is
the same. So under every valid tiling the int64 density must equal the oracle's bit for bit and the force must meet
the same bar as the default tiling (relative L2 2e-5, max 2e-4 of the largest component), and the batched form must
still equal its own single-box runs. Each test restores the built-in tiling when it ends.
"""
import itertools
import json

import numpy as np
import pytest

import synth
from oracle import pm as opm
from tests.gpu_util import rel_l2, requires_gpu, say, to_dev, to_np, torch

pytestmark = [pytest.mark.gpu, requires_gpu]


@pytest.fixture(autouse=True)
def builtin_tiling_after():
    yield
    from paper_1506_03737_amd import lpc
    lpc.lpc_fft_tiling_reset()


def all_tilings(lpc, nm):
    from paper_1506_03737_amd import autotune
    c = autotune.candidates(nm)
    fields = list(autotune.FIELDS)
    return [dict(zip(fields, combo)) for combo in itertools.product(*(c[f] for f in fields))]


def force(lpc, pos_d, nm, box, want_density=True):
    n = pos_d.shape[1]
    geom = lpc.geometry(0, nm, box)
    ws = lpc.workspace(geom, lpc.LPC_OP_PM_FORCE, n_particles=n)
    grad = torch.empty((3, n), dtype=torch.float32, device="cuda")
    dens = torch.empty((nm, nm, nm), dtype=torch.int64, device="cuda") if want_density else None
    lpc.lpc_pm_force(geom, lpc.stepping(), pos_d, grad, ws, density_out=dens)
    return to_np(grad), (to_np(dens) if want_density else None)


def test_every_tiling_matches_oracle_small_mesh():
    """All 81 tilings of a 48^3 mesh (clustered particles) against the FP64 oracle."""
    from paper_1506_03737_amd import lpc
    nm, box = 48, 300.0
    pos = synth.clustered_positions(2, 30001, box)
    ref_C = opm.deposit_fixed(pos, nm, box)
    ref = opm.pm_force(pos.astype(np.float64), nm, box, deconv_power=1)
    pos_d = to_dev(pos)
    tilings = all_tilings(lpc, nm)
    say(f"tiling: {len(tilings)} tilings at nm={nm}")
    assert len(tilings) == 81
    bitwise = 0
    g0 = None
    for t in tilings:
        lpc.lpc_fft_tiling_set(nm, t)
        assert lpc.lpc_fft_tiling_get(nm) == t
        g, d = force(lpc, pos_d, nm, box)
        assert np.array_equal(d, ref_C), t
        assert rel_l2(g, ref) < 2e-5, t
        assert np.abs(g - ref).max() < 2e-4 * np.abs(ref).max(), t
        if g0 is None:
            g0 = g
        bitwise += int(np.array_equal(g, g0))
    say(f"  forces bitwise equal to the first tiling's: {bitwise} of {len(tilings)}")


@pytest.mark.parametrize("nm", [96, 384])
def test_every_tiling_matches_builtin(nm):
    """Every tiling of a larger mesh against the built-in tiling's result (same particles)."""
    from paper_1506_03737_amd import lpc
    box = 500.0
    pos_d = to_dev(synth.clustered_positions(5, 200003, box))
    g_ref, d_ref = force(lpc, pos_d, nm, box)
    tilings = all_tilings(lpc, nm)
    say(f"tiling: {len(tilings)} tilings at nm={nm}")
    for t in tilings:
        lpc.lpc_fft_tiling_set(nm, t)
        g, d = force(lpc, pos_d, nm, box)
        assert np.array_equal(d, d_ref), t
        assert rel_l2(g, g_ref) < 2e-6, t
        assert np.abs(g - g_ref).max() < 2e-5 * np.abs(g_ref).max(), t


@pytest.mark.parametrize("nm", [192, 256, 320])
def test_chained_x_pass_matches_oracle(nm):
    """At the x plans 8 8 R (192, 256, 320) the fused x pass chains its three transforms through registers when its
    tiles are 8 columns wide (the width the autotuner picks there); the built-in 16-column tiles take the unchained
    form. Both against the FP64 oracle (density bit for bit, force at the standard bars) and against each other."""
    from paper_1506_03737_amd import lpc
    box = 400.0
    pos = synth.clustered_positions(7, 150001, box)
    ref_C = opm.deposit_fixed(pos, nm, box)
    ref = opm.pm_force(pos.astype(np.float64), nm, box, deconv_power=1)
    pos_d = to_dev(pos)
    say(f"tiling: chained and unchained fused x pass at nm={nm}")
    out = {}
    for w in (16, 8):
        lpc.lpc_fft_tiling_set(nm, dict(lpc.lpc_fft_tiling_default(nm), poisson_cols=w))
        g, d = force(lpc, pos_d, nm, box)
        assert np.array_equal(d, ref_C), w
        assert rel_l2(g, ref) < 2e-5, w
        assert np.abs(g - ref).max() < 2e-4 * np.abs(ref).max(), w
        out[w] = g
    assert rel_l2(out[8], out[16]) < 2e-6
    assert np.abs(out[8] - out[16]).max() < 2e-5 * np.abs(out[16]).max()


@pytest.mark.parametrize("nm", [768, 1024])
def test_chained_x_pass_matches_unchained_full_size(nm):
    """At the full meshes the fused x pass runs chained through registers on 8-column tiles (plans 8 8 12 and
    4 4 8 8, the latter with two butterflies per thread in its register stages) and unchained on 4-column tiles.
    The two forms share no transform code beyond the butterflies: forces on 2M clustered particles agree to FP32
    rounding, and the density is the same bits."""
    from paper_1506_03737_amd import lpc
    box = 1000.0 if nm == 768 else 2000.0
    pos_d = to_dev(synth.clustered_positions(8, 2000003, box))
    say(f"tiling: chained (8 columns) and unchained (4 columns) fused x pass at nm={nm}")
    out = {}
    for w in (4, 8):
        lpc.lpc_fft_tiling_set(nm, dict(lpc.lpc_fft_tiling_default(nm), poisson_cols=w))
        out[w] = force(lpc, pos_d, nm, box)
    assert np.array_equal(out[4][1], out[8][1])
    g4, g8 = out[4][0], out[8][0]
    say(f"  rel L2 {rel_l2(g8, g4):.3e}, max {np.abs(g8 - g4).max() / np.abs(g4).max():.3e} of max")
    assert rel_l2(g8, g4) < 2e-6
    assert np.abs(g8 - g4).max() < 2e-5 * np.abs(g4).max()


def test_fft_round_trip_under_other_tilings():
    """lpc_fft_r2c / lpc_fft_c2r use z_rows and axis_cols: every fitting pair against numpy.fft."""
    from paper_1506_03737_amd import autotune, lpc
    n = 96
    f = np.random.default_rng(3).standard_normal((n, n, n)).astype(np.float32)
    ref = np.fft.rfftn(f.astype(np.float64))
    c = autotune.candidates(n)
    geom = lpc.geometry(0, n, 1.0)
    ws = lpc.workspace(geom, lpc.LPC_OP_FFT)
    pitch = lpc.lpc_fft_pitch(n)
    for zr, ac in itertools.product(c["z_rows"], c["axis_cols"]):
        t = dict(lpc.lpc_fft_tiling_default(n), z_rows=zr, axis_cols=ac)
        lpc.lpc_fft_tiling_set(n, t)
        spec = torch.empty((n, n, pitch, 2), dtype=torch.float32, device="cuda")
        lpc.lpc_fft_r2c(n, to_dev(f), spec, ws)
        s = to_np(spec)
        got = s[..., : n // 2 + 1, 0] + 1j * s[..., : n // 2 + 1, 1]
        assert rel_l2(got, ref) < 1e-6, t
        back = torch.empty((n, n, n), dtype=torch.float32, device="cuda")
        lpc.lpc_fft_c2r(n, spec, back, ws)
        assert np.abs(to_np(back) / n**3 - f).max() < 1e-5 * np.abs(f).max(), t


def test_batched_graph_rerecorded_after_tiling_change():
    """A batched call replays its recorded graph; after a tiling change the next call records a new one. Both results
    equal the single-box runs of the same boxes."""
    from paper_1506_03737_amd import lpc
    cosmo = lpc.cosmology(**synth.COSMOLOGY)
    step = lpc.stepping(**synth.STEPPING)
    a_list = np.linspace(0.1, 1.0, 4)
    boxes = [(32, 64, 200.0, 11), (48, 96, 300.0, 12), (40, 80, 250.0, 13)]
    ics = []
    for n, nm, box, seed in boxes:
        g = lpc.geometry(n, nm, box)
        ps = lpc.ParticleSet.empty(n**3, "cuda")
        lpc.lpc_init_ic(g, cosmo, seed, a_list[0], ps, lpc.workspace(g, lpc.LPC_OP_INIT_IC))
        ics.append(ps)

    def clone(ps):
        return lpc.ParticleSet(*(torch.clone(getattr(ps, k)) for k in ("pos", "vel", "psi1", "psi2", "id")))

    singles = []
    for (n, nm, box, _), ic in zip(boxes, ics):
        ps = clone(ic)
        g = lpc.geometry(n, nm, box)
        lpc.lpc_cola_step(g, cosmo, step, a_list, ps, lpc.workspace(g, lpc.LPC_OP_COLA_STEP))
        singles.append((to_np(ps.pos), to_np(ps.vel)))

    def batched():
        sets = [clone(ic) for ic in ics]
        entries = [(lpc.geometry(n, nm, box), ps) for (n, nm, box, _), ps in zip(boxes, sets)]
        ws = lpc.workspace_batched(entries)
        lpc.lpc_cola_step_batched(entries, cosmo, step, a_list, ws)
        for ps, ic in zip(sets, ics):  # back to the initial conditions; the second call replays the graph
            for k in ("pos", "vel", "psi1", "psi2", "id"):
                getattr(ps, k).copy_(getattr(ic, k))
        lpc.lpc_cola_step_batched(entries, cosmo, step, a_list, ws)
        return [(to_np(ps.pos), to_np(ps.vel)) for ps in sets]

    lpc.lpc_graph_enable(True)
    say("tiling: batched graph before and after a tiling change")
    first = batched()
    for nm in (64, 80, 96):
        lpc.lpc_fft_tiling_set(nm, dict(z_rows=8, axis_cols=8, poisson_cols=4, c2r_rows=4))
    second = batched()
    for (sp, sv), (p1, v1), (p2, v2) in zip(singles, first, second):
        for a, b in ((p1, sp), (v1, sv), (p2, sp), (v2, sv)):
            assert np.array_equal(a, b)


def test_autotune_sets_and_caches(tmp_path):
    """tune() picks a fitting width per pass, sets it, and the JSON cache gives it back after a reset."""
    from paper_1506_03737_amd import autotune, lpc
    nm = 128
    res = autotune.tune(nm, "cuda", reps=2, log=say)
    cands = autotune.candidates(nm)
    for f in autotune.FIELDS:
        assert res["tiling"][f] in cands[f]
        assert len(res["stage_ms"][f]) == len(cands[f])
    assert lpc.lpc_fft_tiling_get(nm) == res["tiling"]
    path = str(tmp_path / "tiling.json")
    arch = autotune.arch_name()
    autotune.save(path, [res], arch)
    lpc.lpc_fft_tiling_reset()
    assert autotune.apply(path, arch) == [nm]
    assert lpc.lpc_fft_tiling_get(nm) == res["tiling"]
    with open(path) as fh:
        assert json.load(fh)[arch][str(nm)] == res["tiling"]
