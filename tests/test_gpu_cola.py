"""GPU parity of the full COLA run (lpc_cola_step) against the FP64 oracle, fed the same FP32 initial conditions.

Bar: particle positions within 1e-5 L of the oracle after ten steps (periodic minimal image, max over particles);
velocities within 1e-4 of their rms. FP32 positions carry an ulp of 1.5e-5 Mpc/h at 256 Mpc/h, so ten drifts and
the FP32 force error (~1e-6 relative) stay two orders of magnitude inside the bar.
"""
import numpy as np
import pytest

import synth
from oracle import cola as ocola
from oracle import ic as oic
from tests.gpu_util import particle_set, periodic_diff, requires_gpu, say, to_np, torch

pytestmark = [pytest.mark.gpu, requires_gpu]

C = synth.COSMOLOGY


def small_ic(seed=1, n_side=32, box=256.0):
    init = oic.initial_conditions(seed, n_side, box, synth.A_LIST[0], **C)
    return {k: init[k].astype(np.float32) for k in ("pos", "vel", "psi1", "psi2")}


def gpu_run(lpc, ic32, a_list, n_side, nm, box, **step):
    ps = particle_set(lpc, ic32["pos"], ic32["vel"], ic32["psi1"], ic32["psi2"])
    geom = lpc.geometry(n_side, nm, box)
    ws = lpc.workspace(geom, lpc.LPC_OP_COLA_STEP)
    lpc.lpc_cola_step(geom, lpc.cosmology(**C), lpc.stepping(**step), a_list, ps, ws)
    return to_np(ps.pos), to_np(ps.vel)


def oracle_run(ic32, a_list, nm, box, **step):
    kw = {"cola": bool(step.get("cola", 1)), "modified": bool(step.get("modified", 1)),
          "n_lpt": step.get("n_lpt", -2.5), "deconv_power": step.get("deconv_power", 1)}
    return ocola.cola_run(ic32["pos"], ic32["vel"], ic32["psi1"], ic32["psi2"], a_list, C["omega_m"], nm, box, **kw)


@pytest.mark.parametrize("seed", [1, 2])
def test_small_workload_ten_steps(seed):
    """32^3 particles, 64^3 mesh, 256 Mpc/h, ten modified-COLA steps from z = 9 to 0."""
    from paper_1506_03737_amd import lpc
    say(f"cola: small workload seed={seed}")
    box = 256.0
    ic32 = small_ic(seed)
    x, v = gpu_run(lpc, ic32, synth.A_LIST, 32, 64, box)
    xr, vr = oracle_run(ic32, synth.A_LIST, 64, box)
    dx = np.abs(periodic_diff(x, xr, box)).max() / box
    dv = np.sqrt(np.mean((v - vr) ** 2)) / np.sqrt(np.mean(vr**2))
    say(f"  max |dx|/L = {dx:.3e}, rms |dv|/rms v = {dv:.3e}")
    assert dx < 1e-5
    assert dv < 1e-4


@pytest.mark.parametrize("step", [dict(cola=0, modified=0), dict(cola=1, modified=0), dict(cola=1, deconv_power=2),
                                  dict(cola=0, modified=1, deconv_power=0)],
                         ids=["pm-standard", "cola-standard", "cola-deconv2", "pm-modified-nodeconv"])
def test_stepping_variants(step):
    from paper_1506_03737_amd import lpc
    say(f"cola: variant {step}")
    box = 256.0
    ic32 = small_ic(3)
    a = synth.A_LIST
    x, v = gpu_run(lpc, ic32, a, 32, 64, box, **step)
    xr, vr = oracle_run(ic32, a, 64, box, **step)
    d = np.abs(periodic_diff(x, xr, box)) / box
    say(f"  max |dx|/L = {d.max():.3e}, rms = {np.sqrt(np.mean(d**2)):.3e}")
    if step.get("deconv_power", 1) == 2:
        # Dividing by W^2 amplifies the mesh-corner modes by up to (pi/2)^12 ~ 226, so FP32 rounding in the force
        # grows ~15x faster than with one window; the bar scales accordingly (still a small fraction of a cell).
        assert d.max() < 3e-5 and np.sqrt(np.mean(d**2)) < 2e-6
    else:
        assert d.max() < 1e-5


def test_ragged_mesh_and_count():
    """A mesh that is not a power of two (Nm = 96 = 3 x 32) and Nm = 3N, with the 48^3 lattice."""
    from paper_1506_03737_amd import lpc
    say("cola: N=32, Nm=96")
    box = 256.0
    ic32 = small_ic(4)
    a = synth.A_LIST[:6]
    x, v = gpu_run(lpc, ic32, a, 32, 96, box)
    xr, vr = oracle_run(ic32, a, 96, box)
    assert np.abs(periodic_diff(x, xr, box)).max() / box < 1e-5


def test_deterministic_and_resumable():
    from paper_1506_03737_amd import lpc
    say("cola: determinism and resume")
    box = 256.0
    ic32 = small_ic(5)
    a = synth.A_LIST
    x1, v1 = gpu_run(lpc, ic32, a, 32, 64, box)
    x2, v2 = gpu_run(lpc, ic32, a, 32, 64, box)
    assert np.array_equal(x1, x2) and np.array_equal(v1, v2)
    xa, va = gpu_run(lpc, ic32, a[:6], 32, 64, box)
    mid = dict(ic32, pos=xa, vel=va)
    xb, vb = gpu_run(lpc, mid, a[5:], 32, 64, box)
    assert np.abs(periodic_diff(xb, x1, box)).max() / box < 1e-5
    assert np.sqrt(np.mean((vb - v1) ** 2)) < 1e-4 * np.sqrt(np.mean(v1**2))


def test_plane_wave_zeldovich_on_gpu():
    """The exact plane-wave solution: x(a) = q + D1(a) Psi1 (Psi2 = 0); the GPU run matches the oracle's run."""
    from paper_1506_03737_amd import lpc
    from oracle import cosmology as oc
    say("cola: plane wave")
    box, n = 256.0, 32
    q = oic.lattice_positions(n, box)
    psi1 = np.zeros_like(q)
    psi1[0] = 0.5 * box / (2 * np.pi) * np.sin(2 * np.pi * q[0] / box)
    psi2 = np.zeros_like(q)
    a0 = synth.A_LIST[0]
    f1, _ = oc.frame_momentum_factors(a0, C["omega_m"])
    ic32 = {"pos": (q + oc.growth_D1(a0, C["omega_m"]) * psi1).astype(np.float32),
            "vel": (f1 * psi1).astype(np.float32), "psi1": psi1.astype(np.float32), "psi2": psi2.astype(np.float32)}
    x, v = gpu_run(lpc, ic32, synth.A_LIST, n, n, box)
    xr, vr = oracle_run(ic32, synth.A_LIST, n, box)
    assert np.abs(periodic_diff(x, xr, box)).max() / box < 1e-5
    xt = q + psi1
    assert np.abs(periodic_diff(x, xt, box)).max() < 0.15 * box / n


def test_caller_order_is_preserved():
    """The run tile-sorts particles internally and writes them back in the caller's order: a shuffled particle set
    gives the shuffled result of the unshuffled run, bit for bit (integer deposit, per-particle updates)."""
    from paper_1506_03737_amd import lpc
    say("cola: shuffled input order")
    box = 256.0
    ic32 = small_ic(6)
    a = synth.A_LIST[:5]
    x1, v1 = gpu_run(lpc, ic32, a, 32, 64, box)
    perm = np.random.default_rng(6).permutation(32**3)
    shuf = {k: np.ascontiguousarray(v[:, perm]) for k, v in ic32.items()}
    x2, v2 = gpu_run(lpc, shuf, a, 32, 64, box)
    assert np.array_equal(x2, x1[:, perm]) and np.array_equal(v2, v1[:, perm])
