"""GPU parity of the on-the-fly lightcone (lpc_cola_step_lightcone, Sec. 6.1, 6.2) against the FP64 oracle.

Records come in no fixed order and a particle near a box face may sit in one replicate on the GPU and in the next on
the oracle (its wrapped FP32 position just below L, its FP64 one just above 0), so records are matched by particle
and physical position (within 0.05 Mpc/h; images of one particle lie a box length apart). Bars for matched records:
position within 1e-5 L (the run's own position bar), crossing time within 1e-5, momentum within 1e-4 of its rms. A
record without a partner must be a boundary case: its crossing time within 1e-4 of a step end, in units of the step
(the GPU's FP32 distances differ from the oracle's by ~1e-3 Mpc/h, the lightcone moves ~300 Mpc/h per step).
"""
import numpy as np
import pytest

import synth
from oracle import ic as oic
from oracle import lightcone as olc
from tests.gpu_util import particle_set, requires_gpu, say, to_np, torch

pytestmark = [pytest.mark.gpu, requires_gpu]

C = synth.COSMOLOGY


def small_ic(seed, n_side=32, box=256.0):
    init = oic.initial_conditions(seed, n_side, box, synth.A_LIST[0], **C)
    return {k: init[k].astype(np.float32) for k in ("pos", "vel", "psi1", "psi2")}


def gpu_lightcone(lpc, ic32, a_list, n_side, nm, box, origin, a_start, rep_lo, rep_hi, capacity, **step):
    ps = particle_set(lpc, ic32["pos"], ic32["vel"], ic32["psi1"], ic32["psi2"])
    geom = lpc.geometry(n_side, nm, box)
    ws = lpc.workspace(geom, lpc.LPC_OP_COLA_STEP)
    rec = torch.zeros((capacity, lpc.LIGHTCONE_RECORD_FIELDS), dtype=torch.float32, device="cuda")
    lc = lpc.lightcone(origin, a_start, rec, rep_lo, rep_hi)
    count = lpc.lpc_cola_step_lightcone(geom, lpc.cosmology(**C), lpc.stepping(**step), a_list, ps, lc, ws)
    r = to_np(rec[:count])
    ints = r.view(np.int32)
    out = {"pos": r[:, 0:3].T.astype(np.float64), "vel": r[:, 3:6].T.astype(np.float64), "a": r[:, 6].astype(np.float64),
           "index": ints[:, 7].astype(np.int64), "replicate": ints[:, 8].astype(np.int64)}
    return out, to_np(ps.pos), to_np(ps.vel)


def record_keys(rec, R, a_list):
    """(particle, replicate, drift) of each record as one integer. A particle image crosses at most once, but the
    replicate that names it changes when the particle wraps across a box face, so (particle, replicate) alone can
    repeat over the drifts of a run."""
    step = np.clip(np.searchsorted(np.asarray(a_list), rec["a"], side="right") - 1, 0, len(a_list) - 2)
    return (rec["index"] * R + rec["replicate"]) * len(a_list) + step


def match(got, ref, a_list, tol=0.05):
    """Pairs (i_got, i_ref) of records of the same particle within tol of each other; and the unpaired of each.
    Records with the same (particle, replicate, drift) pair up first; the rest are paired by position."""
    R = int(max(got["replicate"].max(initial=0), ref["replicate"].max(initial=0))) + 1
    kg = record_keys(got, R, a_list)
    kr = record_keys(ref, R, a_list)
    assert np.unique(kg).size == kg.size and np.unique(kr).size == kr.size
    _, ig, ir = np.intersect1d(kg, kr, assume_unique=True, return_indices=True)
    close = np.abs(got["pos"][:, ig] - ref["pos"][:, ir]).max(axis=0) < tol
    pairs = [np.stack([ig[close], ir[close]], axis=1)]
    rest_g = np.setdiff1d(np.arange(kg.size), ig[close])
    rest_r = np.setdiff1d(np.arange(kr.size), ir[close])
    by_index = {}
    for j in rest_r.tolist():
        by_index.setdefault(int(ref["index"][j]), []).append(j)
    used, lone_got, extra = set(), [], []
    for i in rest_g.tolist():
        hit = None
        for j in by_index.get(int(got["index"][i]), ()):
            if j not in used and np.abs(got["pos"][:, i] - ref["pos"][:, j]).max() < tol:
                hit = j
                break
        if hit is None:
            lone_got.append(i)
        else:
            used.add(hit)
            extra.append((i, hit))
    pairs.append(np.array(extra, dtype=np.int64).reshape(-1, 2))
    lone_ref = [j for j in rest_r.tolist() if j not in used]
    return np.concatenate(pairs), lone_got, lone_ref


def step_fraction(a, a_list):
    """Position of each crossing time within its step (0 at the start, 1 at the end)."""
    a_list = np.asarray(a_list)
    i = np.clip(np.searchsorted(a_list, a, side="right") - 1, 0, a_list.size - 2)
    return (a - a_list[i]) / (a_list[i + 1] - a_list[i])


def check_against_oracle(got, ref, a_list, box):
    pairs, lone_got, lone_ref = match(got, ref, a_list)
    say(f"  records: GPU {got['a'].size}, oracle {ref['a'].size}, matched {len(pairs)}, unpaired "
        f"{len(lone_got)} / {len(lone_ref)}")
    assert len(pairs) > 0.999 * ref["a"].size
    for recs, lone in ((got, lone_got), (ref, lone_ref)):
        if lone:
            t = step_fraction(recs["a"][lone], a_list)
            assert np.all(np.minimum(t, 1.0 - t) < 1e-4), t
    g, r = pairs[:, 0], pairs[:, 1]
    dx = np.abs(got["pos"][:, g] - ref["pos"][:, r]).max() / box
    da = np.abs(got["a"][g] - ref["a"][r]).max()
    dv = np.sqrt(np.mean((got["vel"][:, g] - ref["vel"][:, r]) ** 2)) / np.sqrt(np.mean(ref["vel"][:, r] ** 2))
    say(f"  matched: max |dx|/L {dx:.3e}, max |da| {da:.3e}, rms |dv|/rms v {dv:.3e}")
    assert dx < 1e-5 and da < 1e-5 and dv < 1e-4
    # the replicate index names the same image, up to the particles at a box face
    same = got["replicate"][g] == ref["replicate"][r]
    assert same.mean() > 0.999


@pytest.mark.parametrize("step", [dict(), dict(cola=0, modified=0)], ids=["cola-modified", "pm-standard"])
def test_lightcone_matches_oracle(step):
    """The small workload (32^3 particles, 64^3 mesh, 256 Mpc/h), observer at the box corner, the lightcone on the last
    two drifts (from a = 0.82, R_L = 623 Mpc/h) through 6 x 6 x 6 replicates: about two million records."""
    from paper_1506_03737_amd import lpc
    say(f"lightcone: small workload, 216 replicates, {step}")
    box, a = 256.0, synth.A_LIST
    ic32 = small_ic(11)
    origin, a_start, lo, hi = (0.0, 0.0, 0.0), a[8], (-3, -3, -3), (2, 2, 2)
    got, x, v = gpu_lightcone(lpc, ic32, a, 32, 64, box, origin, a_start, lo, hi, 3_000_000, **step)
    kw = {"cola": bool(step.get("cola", 1)), "modified": bool(step.get("modified", 1))}
    xr, vr, ref = olc.lightcone_run(ic32["pos"], ic32["vel"], ic32["psi1"], ic32["psi2"], a, C["omega_m"], 64, box,
                                    origin, a_start, lo, hi, **kw)
    check_against_oracle(got, ref, a, box)


def test_lightcone_inside_the_box_observer_and_run_unchanged():
    """Observer inside the box, lightcone from a = 0.91 (R_L = 290 Mpc/h) with 3 x 3 x 3 replicates; the particles at
    the end equal those of lpc_cola_step bit for bit (the lightcone only reads the drift), and a second run gives the
    same records (as a set) bit for bit."""
    from paper_1506_03737_amd import lpc
    say("lightcone: observer inside the box; run unchanged; repeatable")
    box, a = 256.0, synth.A_LIST
    ic32 = small_ic(12)
    origin, lo, hi = (100.0, 130.0, 60.0), (-1, -1, -1), (1, 1, 1)
    got, x, v = gpu_lightcone(lpc, ic32, a, 32, 64, box, origin, a[9], lo, hi, 1_000_000)
    got2, _, _ = gpu_lightcone(lpc, ic32, a, 32, 64, box, origin, a[9], lo, hi, 1_000_000)
    ps = particle_set(lpc, ic32["pos"], ic32["vel"], ic32["psi1"], ic32["psi2"])
    geom = lpc.geometry(32, 64, box)
    lpc.lpc_cola_step(geom, lpc.cosmology(**C), lpc.stepping(), a, ps, lpc.workspace(geom, lpc.LPC_OP_COLA_STEP))
    assert np.array_equal(to_np(ps.pos), x) and np.array_equal(to_np(ps.vel), v)
    key = lambda r: np.lexsort((r["a"], r["replicate"], r["index"]))
    o1, o2 = key(got), key(got2)
    for f in ("index", "replicate", "a"):
        assert np.array_equal(got[f][o1], got2[f][o2])
    assert np.array_equal(got["pos"][:, o1], got2["pos"][:, o2])
    xr, vr, ref = olc.lightcone_run(ic32["pos"], ic32["vel"], ic32["psi1"], ic32["psi2"], a, C["omega_m"], 64, box,
                                    origin, a[9], lo, hi)
    check_against_oracle(got, ref, a, box)


def test_lightcone_capacity_and_errors():
    from paper_1506_03737_amd import lpc
    say("lightcone: capacity and argument errors")
    box, a = 256.0, synth.A_LIST
    ic32 = small_ic(13)
    full, _, _ = gpu_lightcone(lpc, ic32, a, 32, 64, box, (0.0, 0.0, 0.0), a[9], (-1, -1, -1), (1, 1, 1), 500_000)
    n = full["a"].size
    assert n > 1000
    ps = particle_set(lpc, ic32["pos"], ic32["vel"], ic32["psi1"], ic32["psi2"])
    geom = lpc.geometry(32, 64, box)
    ws = lpc.workspace(geom, lpc.LPC_OP_COLA_STEP)
    rec = torch.zeros((100, lpc.LIGHTCONE_RECORD_FIELDS), dtype=torch.float32, device="cuda")
    lc = lpc.lightcone((0.0, 0.0, 0.0), a[9], rec, (-1, -1, -1), (1, 1, 1))
    with pytest.raises(lpc.LpcError) as e:
        lpc.lpc_cola_step_lightcone(geom, lpc.cosmology(**C), lpc.stepping(), a, ps, lc, ws)
    assert e.value.status == -7 and e.value.count == n
    kept = to_np(rec).view(np.int32)[:, 7]
    assert np.all(np.isin(kept, full["index"]))
    bad = lpc.lightcone((0.0, 0.0, 0.0), a[9], rec, (1, 0, 0), (0, 0, 0))
    with pytest.raises(lpc.LpcError) as e:
        lpc.lpc_cola_step_lightcone(geom, lpc.cosmology(**C), lpc.stepping(), a, ps, bad, ws)
    assert e.value.status == -1


def test_full_size_lightcone_properties():
    """The single-box workload (256^3 particles from lpc_init_ic, 768^3 mesh, 1000 Mpc/h) with the observer at the
    box corner, the lightcone on the last two drifts through 2 x 2 x 2 replicates: every record's distance from the
    observer at its crossing time equals the step's linear interpolation of R_L there (the estimate the crossing time
    solves) to within the curvature of the particle's path over a step (0.5 Mpc/h; R_L's own curvature puts the exact
    R_L up to ~5 Mpc/h away at mid-step), crossing times lie in the lightcone drifts, each (particle, replicate, drift)
    occurs at most once, and the final particles equal the plain run's bit for bit."""
    from paper_1506_03737_amd import lpc
    say("lightcone: 256^3 particles, 768^3 mesh, 8 replicates")
    N, nm, box = 256, 768, 1000.0
    n = N**3
    a = synth.A_LIST
    geom = lpc.geometry(N, nm, box)
    ic = lpc.ParticleSet.empty(n)
    ws = lpc.workspace(geom, lpc.LPC_OP_INIT_IC)
    lpc.lpc_init_ic(geom, lpc.cosmology(**C), 2015, a[0], ic, ws)
    del ws
    ws = lpc.workspace(geom, lpc.LPC_OP_COLA_STEP)
    ps = lpc.ParticleSet(*(torch.clone(getattr(ic, k)) for k in ("pos", "vel", "psi1", "psi2", "id")))
    cap = 24_000_000
    rec = torch.zeros((cap, lpc.LIGHTCONE_RECORD_FIELDS), dtype=torch.float32, device="cuda")
    lc = lpc.lightcone((0.0, 0.0, 0.0), a[8], rec, (-1, -1, -1), (0, 0, 0))
    count = lpc.lpc_cola_step_lightcone(geom, lpc.cosmology(**C), lpc.stepping(), a, ps, lc, ws)
    say(f"  {count} records")
    assert count > 1_000_000
    r = rec[:count]
    ints = r.view(torch.int32)
    pos, acr = r[:, 0:3].double(), r[:, 6].double()
    ends = np.array(a[8:])
    r_ends = lpc.lpc_comoving_distance(lpc.cosmology(**C), ends)
    r_l = torch.from_numpy(np.interp(acr.cpu().numpy(), ends, r_ends)).cuda()  # piecewise linear between step ends
    dist = pos.norm(dim=1)
    err = (dist - r_l).abs().max().item()
    say(f"  max |R_p(a_L) - R_L,lin(a_L)| = {err:.4f} Mpc/h")
    assert err < 0.5
    assert float(acr.min()) >= a[8] - 1e-6 and float(acr.max()) <= 1.0
    step = (acr >= a[9]).long()
    key = (ints[:, 7].long() * 8 + ints[:, 8].long()) * 2 + step
    assert torch.unique(key).numel() == count
    plain = lpc.ParticleSet(*(torch.clone(getattr(ic, k)) for k in ("pos", "vel", "psi1", "psi2", "id")))
    lpc.lpc_cola_step(geom, lpc.cosmology(**C), lpc.stepping(), a, plain, ws)
    assert torch.equal(plain.pos, ps.pos) and torch.equal(plain.vel, ps.vel)
