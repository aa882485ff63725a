"""Throughput benchmark of the PM-COLA time step on one MI355X.

Workload (the single-box configuration): 256^3 particles, 768^3 mesh, 1000 Mpc/h box, 2LPT initial conditions at
z = 9 from a seeded BBKS Gaussian field (generated on the GPU by lpc_init_ic, untimed), ten modified-COLA steps
uniform in a from 0.1 to 1.0 (nLPT = -2.5), CIC window deconvolved once.

A "step" is one COLA time step of that ten-step schedule: drift + full PM force (deposit, r2c FFT, Poisson/gradient,
3 c2r, gather) + kick. `--steps K` times K steps as repetitions of the schedule: K // 10 full lpc_cola_step calls
over the 11 scale factors, and, if K is not a multiple of 10, one call over the first K % 10 steps, each started from
the initial conditions (reset untimed) and bracketed by device synchronisations. value = N^3 K / (sum of the call
times) in particle-steps/s, inputs resident in HBM. The timed calls record HIP events around every launch on the
call's stream; those give the per-stage table and the dominant kernel's roofline.

Extras in the same JSON line:
  roofline     the dominant kernel: algorithmic bytes per launch / mean launch time, against the 8 TB/s HBM peak
               and against a device-to-device copy measured here (copy_peak);
  batched      48 uneven boxes (96^3/128^3/160^3 particles, Nm = 2N, L = 300..600 Mpc/h), one recorded HIP graph of
               the ten-step run replayed (aggregate particle-steps/s);
  learned      coarse Nm = N run plus the trained correction network against the fine Nm = 3N run (ten steps);
  large        the large single box (512^3 particles, 1024^3 mesh, 2000 Mpc/h), one ten-step call;
  lightcone    the single box with the on-the-fly lightcone on its last two drifts (observer at a box corner,
               2 x 2 x 2 replicates) against the same run without it;
  cpu_baseline the FP64 oracle on the host: the 32^3 / 64^3 / 256 Mpc/h configuration in full on one core and in one
               process per core, and a two-step sample of the single box at 1/8 volume corrected to the ten-step
               schedule's force evaluations per step;
  precision    the GPU against the oracle on that small configuration after ten steps: positions, momenta, P(k).

Usage: python bench.py [--gpus 1] [--steps 10] [--warmup 1] [--workload single|small|large] [--no-cpu] [--no-batched]
                      [--no-learned] [--no-large] [--no-lightcone] [--no-tune] [--tiling-cache PATH]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "particle-steps/s (COLA PM step), plain vs batched/learned at P(k) err <2%"
HBM_PEAK_GBS = 8000.0


def note(msg):
    """A progress line on stderr (the JSON result is the only line on stdout)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)

# HBM bytes per launch measured with rocprofv3 FETCH_SIZE / WRITE_SIZE passes (read scaled by 2.0, write by 1.0, from
# a 1 GiB copy), by (stage, mesh size, tile width of the stage); profiles/force_path_768_hbm_traffic.md. Must be
# re-measured (or removed) when the kernel changes.
MEASURED_TRAFFIC = {("fft z c2r", 768, 4): 10.985e9, ("fft y inv", 768, 8): 9.292e9, ("fft x + poisson", 768, 8): 5.657e9,
                    ("fft y", 768, 8): 3.796e9, ("fft z r2c", 768, 16): 3.643e9}

# Stages run once per force evaluation: their algorithmic bytes are counted per evaluation and spread over its launches
PER_EVALUATION = ("deposit", "fft z r2c", "fft y", "fft x + poisson", "fft y inv", "fft z c2r", "gather kick drift")


def stage_bytes(stage, n_part, nm):
    """Algorithmic HBM bytes of one launch of each force-path stage, from per-unit figures: a 1-D transform pass over
    the mesh moves 8 B per cell (read and write of the half spectrum),
    and a launch counts each transform it performs; the CIC deposit moves 12 B per particle and 8 B per cell; the
    gather + kick + drift reads the force mesh (12 B per cell) and 48 B of particle state and writes 24 B (plus the
    next sort's key and rank, 8 B) per particle."""
    M = nm**3
    return {
        "deposit": 12 * n_part + 8 * M,
        "fft z r2c": 8 * M,                 # one transform
        "fft y": 8 * M,                     # one transform
        "fft x + poisson": 3 * 8 * M,       # forward x, inverse x of the x gradient, inverse x of the potential
        "fft y inv": 3 * 8 * M,             # x gradient, i k_y psi, psi
        "fft z c2r": 3 * 8 * M,             # three components
        "gather kick drift": 80 * n_part + 12 * M,
        "frame velocity": 48 * n_part,      # read vel, psi1, psi2; write vel
    }.get(stage)


def moved_bytes(stage, n_part, nm):
    """The bytes each fused kernel must move at least (FP32 mesh and contrast, half spectra of nm nm (nm/2 + 1)
    complex values): less than stage_bytes where a launch shares loads between transforms."""
    M = nm**3
    H = nm * nm * (nm // 2 + 1) * 8        # bytes of one half-spectrum complex mesh
    return {
        "deposit": 12 * n_part + 4 * M,     # read positions, the FP32 density contrast written once
        "fft z r2c": 4 * M + H,             # read the FP32 contrast, write half spectrum
        "fft y": 2 * H,
        "fft x + poisson": H + 2 * H,       # read delta_hat, write the x gradient and the potential
        "fft y inv": 2 * H + 3 * H,         # x gradient in place; read the potential, write its y gradient and itself
        "fft z c2r": 3 * H + 12 * M,        # read three spectra, write the AoS float3 force mesh
        "gather kick drift": 80 * n_part + 12 * M,
        "frame velocity": 48 * n_part,
    }.get(stage)


def launch_share(name, launches, evals):
    """The fraction of one evaluation's bytes that one launch of a stage moves (1 for a stage launched per call)."""
    return evals / launches if name in PER_EVALUATION else 1.0


def stage_table(stats, n_part, nm, wall_ms, evals, copy_gbs=None):
    stages = {}
    for name, (launches, ms) in stats.items():
        b = stage_bytes(name, n_part, nm)
        avg = ms / launches
        entry = {"launches": launches, "avg_ms": round(avg, 4), "share": round(ms / wall_ms, 4)}
        if name in PER_EVALUATION:
            entry["ms_per_evaluation"] = round(ms / evals, 4)
        if b is not None:
            f = launch_share(name, launches, evals)
            gbs = b * f / (avg * 1e-3) / 1e9
            entry["GB_per_s"] = round(gbs, 1)
            entry["frac_of_8TBs"] = round(gbs / HBM_PEAK_GBS, 4)
            if copy_gbs:
                entry["frac_of_copy"] = round(gbs / copy_gbs, 4)
            mb = moved_bytes(name, n_part, nm)
            entry["moved_GB_per_s"] = round(mb * f / (avg * 1e-3) / 1e9, 1)
        stages[name] = entry
    return stages


def schedule_runs(k):
    """Step counts of the calls that make up k steps of the ten-step schedule."""
    return [10] * (k // 10) + ([k % 10] if k % 10 else [])


def timed_schedule(lpc, torch, geom, cosmo, step, a_list, ps, ws, reset, k, profile):
    """k steps as calls over the ten-step schedule, each reset (untimed) and bracketed by synchronisations; returns
    the summed call time (s) and, with profile, the per-stage event statistics of the timed calls."""
    total = 0.0
    if profile:
        lpc.lpc_profile_reset()
        lpc.lpc_profile_enable(True)
    try:
        for m in schedule_runs(k):
            reset()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            lpc.lpc_cola_step(geom, cosmo, step, a_list[: m + 1], ps, ws)
            torch.cuda.synchronize()
            total += time.perf_counter() - t0
    finally:
        if profile:
            lpc.lpc_profile_enable(False)
    return total, (lpc.lpc_profile_stats() if profile else None)


def copy_peak(torch, nbytes=2 << 30, reps=5):
    """Device-to-device copy bandwidth (bytes read + written / time), best of `reps` copies of nbytes."""
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = None
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(src)
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b)
        best = ms if best is None else min(best, ms)
    del src, dst
    torch.cuda.empty_cache()
    return 2.0 * nbytes / (best * 1e-3) / 1e9


def make_ic(lpc, torch, n_side, box, seed, cosmo):
    n = n_side**3
    geom = lpc.geometry(n_side, n_side, box)
    ic = lpc.ParticleSet.empty(n, "cuda")
    ws = lpc.workspace(geom, lpc.LPC_OP_INIT_IC, "cuda")
    lpc.lpc_init_ic(geom, cosmo, seed, 0.1, ic, ws)
    del ws
    return ic


def batched_bench(lpc, synth, torch):
    """The 48-box batched form over the ten-step schedule: ICs per box (untimed), one recording call, then one timed
    replay of the graph; per-stage times from one more direct-launch run."""
    cosmo = lpc.cosmology(**synth.COSMOLOGY)
    step = lpc.stepping(**synth.STEPPING)
    boxes = synth.batch_workload()
    ics, sets, entries = [], [], []
    for b in boxes:
        ic = make_ic(lpc, torch, b["n_side"], b["box"], b["seed"], cosmo)
        ps = lpc.ParticleSet.empty(b["n_side"] ** 3, "cuda")
        ics.append(ic)
        sets.append(ps)
        entries.append((lpc.geometry(b["n_side"], b["n_mesh"], b["box"]), ps))
    ws = lpc.workspace_batched(entries, "cuda")
    n_total = sum(b["n_side"] ** 3 for b in boxes)

    def reset():
        for ps, ic in zip(sets, ics):
            for k in ("pos", "vel", "psi1", "psi2", "id"):
                getattr(ps, k).copy_(getattr(ic, k))

    a_list = synth.A_LIST
    steps = len(a_list) - 1
    reset()
    lpc.lpc_cola_step_batched(entries, cosmo, step, a_list, ws)  # records the graph (untimed)
    reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lpc.lpc_cola_step_batched(entries, cosmo, step, a_list, ws)  # replays it
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    reset()
    lpc.lpc_profile_reset()
    lpc.lpc_profile_enable(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lpc.lpc_cola_step_batched(entries, cosmo, step, a_list, ws)
    torch.cuda.synchronize()
    dt_prof = time.perf_counter() - t1
    lpc.lpc_profile_enable(False)
    stats = lpc.lpc_profile_stats()
    stages = {}
    for name, (launches, ms) in stats.items():
        per = [stage_bytes(name, b["n_side"] ** 3, b["n_mesh"]) for b in boxes]
        avg = ms / launches
        entry = {"launches": launches, "avg_ms": round(avg, 4), "share": round(ms / (dt_prof * 1e3), 4)}
        if per[0] is not None:
            entry["GB_per_s"] = round(sum(per) / (avg * 1e-3) / 1e9, 1)
        stages[name] = entry
    return {"value": n_total * steps / dt, "unit": "particle-steps/s", "ms_per_step": dt * 1e3 / steps,
            "steps": steps, "boxes": len(boxes), "particles": n_total,
            "workload": "48 boxes, N in {96,128,160} cycling, Nm = 2N, L = 300 + 300 j/47 Mpc/h, seeds 1000 + j, "
                        "2LPT ICs at z=9, ten modified-COLA steps nLPT=-2.5; one graph replay (graph recorded by an "
                        "untimed identical call)",
            "stages_direct_launch": stages}


def learned_bench(lpc, synth, torch):
    """The learned form over the ten-step schedule: a coarse run (Nm = N) plus one network pass, against the fine run
    (Nm = 3N) it stands in for. Training data: 256 coarse/fine pairs of 128^3 particles in 500 Mpc/h boxes (seeds
    5000..5255) made by lpc_cola_step, 8 more held out (seeds 6000..6007); 24 epochs of Adam (lr 1e-3 -> 5e-5,
    cosine), random cube symmetries; the output gain calibrated on the held-out pairs' P(k). Applied to the single-box
    workload (256^3 particles, 1000 Mpc/h, seed 2015): coarse Nm = 256 + network vs fine Nm = 768. Throughput counts
    the coarse run and the network pass; P(k) errors are against the fine run, k <= 0.5 h/Mpc."""
    import numpy as np
    from paper_1506_03737_amd import learned
    dev = torch.device("cuda:0")
    cosmo = lpc.cosmology(**synth.COSMOLOGY)
    step = lpc.stepping(**synth.STEPPING)
    a_list = synth.A_LIST
    steps = len(a_list) - 1
    fit = learned.fit_correction(range(5000, 5256), range(6000, 6008), 128, 500.0, a_list, cosmo, step, dev,
                                 epochs=24)
    params = fit["params"]
    N, box = 256, 1000.0
    n = N**3
    ic = make_ic(lpc, torch, N, box, 2015, cosmo)
    runs = {}
    for name, nm in (("coarse", N), ("fine", 3 * N)):
        ps = lpc.ParticleSet(*(torch.clone(getattr(ic, k)) for k in ("pos", "vel", "psi1", "psi2", "id")))
        geom = lpc.geometry(N, nm, box)
        wsr = lpc.workspace(geom, lpc.LPC_OP_COLA_STEP, dev)
        _, dt = learned.timed(lambda: lpc.lpc_cola_step(geom, cosmo, step, a_list, ps, wsr))
        del wsr
        runs[name] = (ps, dt)
    corrected = lpc.ParticleSet(torch.clone(runs["coarse"][0].pos), None, ic.psi1, None, ic.id)
    ws_net = lpc.net_workspace(N, dev)
    _, t_apply = learned.timed(lambda: lpc.lpc_net_apply(lpc.geometry(N, N, box), params, corrected, ws_net))
    fine = runs["fine"][0].pos
    t_learned = runs["coarse"][1] + t_apply
    # reduced bispectrum (128^3 estimator mesh, shells of 3 kf): equilateral and k2 = 2 k1 triangles
    tri = [(0.05, 0.05, 0.05), (0.1, 0.1, 0.1), (0.2, 0.2, 0.2), (0.3, 0.3, 0.3), (0.1, 0.2, 0.15), (0.1, 0.2, 0.25)]
    gq = lpc.geometry(0, 128, box)
    wsq = lpc.workspace(gq, lpc.LPC_OP_BISPECTRUM, dev, n_particles=n)
    q = {name: lpc.lpc_bispectrum(gq, pos, tri, 3 * 2 * np.pi / box, wsq)[1]
         for name, pos in (("fine", fine), ("coarse", runs["coarse"][0].pos), ("coarse+net", corrected.pos))}
    del wsq
    return {"value": n * steps / t_learned, "unit": "particle-steps/s", "ms_per_step": t_learned * 1e3 / steps,
            "steps": steps, "fine_value": n * steps / runs["fine"][1], "speedup_vs_fine": runs["fine"][1] / t_learned,
            "coarse_run_ms": runs["coarse"][1] * 1e3, "net_apply_ms": t_apply * 1e3, "fine_run_ms": runs["fine"][1] * 1e3,
            "pk_max_rel_err_k_le_0.5": {"coarse": learned.pk_max_error(runs["coarse"][0].pos, fine, n, box, dev),
                                        "coarse+net": learned.pk_max_error(corrected.pos, fine, n, box, dev)},
            "q_rel_err": {name: [round(float(abs(a / b - 1.0)), 5) for a, b in zip(q[name], q["fine"])]
                          for name in ("coarse", "coarse+net")},
            "q_triangles": tri, "q_fine": [round(float(x), 5) for x in q["fine"]],
            "output_gain": fit["gain"], "held_out_pk_err_by_gain": fit["gain_errors"],
            "validation_loss_ratio": fit["validation_loss_ratio"], "train_s": fit["train_s"],
            "pairs_s": fit["pairs_s"], "calibrate_s": fit["calibrate_s"],
            "workload": "256^3 particles, 1000 Mpc/h, seed 2015, ten steps: coarse Nm=256 + network vs fine Nm=768; "
                        "network trained on 256 pairs of 128^3 / 500 Mpc/h (coarse Nm=128, fine Nm=384), 24 epochs, "
                        "output gain calibrated on 8 held-out pairs"}


def large_bench(lpc, synth, torch, copy_gbs):
    """The large single box: 512^3 particles, 1024^3 mesh, 2000 Mpc/h, one ten-step call (untimed warm-up call first),
    with per-stage events."""
    w = synth.WORKLOADS["large"]
    cosmo = lpc.cosmology(**synth.COSMOLOGY)
    step = lpc.stepping(**synth.STEPPING)
    N, nm, box = w["n_side"], w["n_mesh"], w["box"]
    n = N**3
    ic = make_ic(lpc, torch, N, box, w["seed"], cosmo)
    geom = lpc.geometry(N, nm, box)
    ps = lpc.ParticleSet.empty(n, "cuda")
    ws = lpc.workspace(geom, lpc.LPC_OP_COLA_STEP, "cuda")

    def reset():
        for k in ("pos", "vel", "psi1", "psi2", "id"):
            getattr(ps, k).copy_(getattr(ic, k))

    timed_schedule(lpc, torch, geom, cosmo, step, synth.A_LIST, ps, ws, reset, 1, False)
    dt, stats = timed_schedule(lpc, torch, geom, cosmo, step, synth.A_LIST, ps, ws, reset, 10, True)
    stages = stage_table(stats, n, nm, dt * 1e3, sum(m + 1 for m in schedule_runs(10)), copy_gbs)
    del ps, ws, ic
    torch.cuda.empty_cache()
    return {"value": n * 10 / dt, "unit": "particle-steps/s", "ms_per_step": dt * 1e3 / 10, "steps": 10,
            "workload": f"large: {N}^3 particles, {nm}^3 mesh, {box:g} Mpc/h, 2LPT ICs at z=9, ten modified-COLA steps",
            "stages": stages}


def lightcone_bench(lpc, synth, torch, ic, geom, ws, n):
    """The single box with the lightcone on its last two drifts (from a = 0.82, R_L = 623 Mpc/h), observer at a box
    corner, replicates covering the sphere (2 x 2 x 2): one ten-step call against a plain one."""
    cosmo = lpc.cosmology(**synth.COSMOLOGY)
    step = lpc.stepping(**synth.STEPPING)
    ps = lpc.ParticleSet(*(torch.clone(getattr(ic, k)) for k in ("pos", "vel", "psi1", "psi2", "id")))
    cap = 24_000_000
    rec = torch.empty((cap, lpc.LIGHTCONE_RECORD_FIELDS), dtype=torch.float32, device="cuda")
    lc = lpc.lightcone((0.0, 0.0, 0.0), synth.A_LIST[8], rec, (-1, -1, -1), (0, 0, 0))

    def reset():
        for k in ("pos", "vel", "psi1", "psi2", "id"):
            getattr(ps, k).copy_(getattr(ic, k))

    times = {}
    for name in ("lightcone", "plain"):
        reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if name == "lightcone":
            count = lpc.lpc_cola_step_lightcone(geom, cosmo, step, synth.A_LIST, ps, lc, ws)
        else:
            lpc.lpc_cola_step(geom, cosmo, step, synth.A_LIST, ps, ws)
        torch.cuda.synchronize()
        times[name] = time.perf_counter() - t0
    del rec, ps
    torch.cuda.empty_cache()
    return {"value": n * 10 / times["lightcone"], "unit": "particle-steps/s", "records": count,
            "run_ms": times["lightcone"] * 1e3, "plain_run_ms": times["plain"] * 1e3,
            "overhead": times["lightcone"] / times["plain"] - 1.0,
            "workload": "single box, lightcone on the last two drifts (a >= 0.82), observer at (0, 0, 0), "
                        "replicates -1..0 per axis"}


def _oracle_small_run(_=None):
    """The oracle's ten-step run of the small configuration (seed 1) from its FP32 initial conditions; returns
    (seconds, pos, vel, ic32)."""
    import numpy as np

    import synth
    from oracle import cola as ocola
    from oracle import ic as oic
    w = synth.WORKLOADS["small"]
    init = oic.initial_conditions(w["seed"], w["n_side"], w["box"], synth.A_LIST[0], **synth.COSMOLOGY)
    ic32 = {k: init[k].astype(np.float32) for k in ("pos", "vel", "psi1", "psi2")}
    t0 = time.perf_counter()
    x, v = ocola.cola_run(ic32["pos"], ic32["vel"], ic32["psi1"], ic32["psi2"], synth.A_LIST,
                          synth.COSMOLOGY["omega_m"], w["n_mesh"], w["box"])
    return time.perf_counter() - t0, x, v, ic32


def cpu_baseline(workers):
    """The FP64 oracle, untuned, on the host (run before the GPU is touched, so the worker processes are plain forks
    of a process without a GPU context). Returns (cpu_baseline object, oracle results for the precision object)."""
    import concurrent.futures
    import multiprocessing
    import platform

    import synth
    from oracle import cola as ocola
    from oracle import ic as oic
    from oracle import pm as opm
    from oracle import spectrum as ospec
    w = synth.WORKLOADS["small"]
    n_small = w["n_side"] ** 3
    t1, x_ref, v_ref, ic32 = _oracle_small_run()
    ctx = multiprocessing.get_context("fork")
    t_all0 = time.perf_counter()
    with concurrent.futures.ProcessPoolExecutor(max_workers=workers, mp_context=ctx) as ex:
        per = [r[0] for r in ex.map(_oracle_small_run, range(workers))]
    t_all = time.perf_counter() - t_all0
    # the single box at 1/8 volume (128^3 particles, 384^3 mesh, 500 Mpc/h): two steps (3 force evaluations, 2 drifts)
    # and one more force evaluation timed alone, to re-weight to the ten-step schedule's 1.1 forces per step
    n_side, nm, box = 128, 384, 500.0
    init = oic.initial_conditions(7, n_side, box, 0.1, **synth.COSMOLOGY)
    t0 = time.perf_counter()
    ocola.cola_run(init["pos"], init["vel"], init["psi1"], init["psi2"], synth.A_LIST[:3],
                   synth.COSMOLOGY["omega_m"], nm, box)
    t_two = time.perf_counter() - t0
    t0 = time.perf_counter()
    opm.pm_force(init["pos"], nm, box, 1)
    t_force = time.perf_counter() - t0
    t_rest = max(0.0, (t_two - 3 * t_force) / 2)          # kick + drift per step
    t_step = 1.1 * t_force + t_rest                         # a step of the ten-step schedule
    k_ref, p_ref, _ = ospec.power_spectrum(x_ref, w["n_mesh"], w["box"], 0.5, 20)
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        model = platform.processor() or "unknown"
    out = {"value": n_small * 10 / t1, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
           "sample": f"FP64 NumPy oracle, the small configuration (32^3 particles, 64^3 mesh, 256 Mpc/h) in full: ten "
                     f"modified-COLA steps in {t1:.2f} s on one core",
           "all_cores": {"value": n_small * 10 * workers / max(per), "unit": "particle-steps/s",
                         "processes": workers, "pool_seconds": round(t_all, 2),
                         "per_process_s": [round(p, 2) for p in per],
                         "sample": "the same ten-step run in one process per core at once (independent realisations); "
                                   "rate over the slowest process's stepping time"},
           "single_box_sample": {"value": n_side**3 / t_step, "unit": "particle-steps/s", "cores": 1,
                                 "two_step_s": round(t_two, 2), "force_s": round(t_force, 2),
                                 "sample": "128^3 particles, 384^3 mesh, 500 Mpc/h (the single box at 1/8 volume): two "
                                           "steps and one force evaluation, re-weighted to 1.1 force evaluations "
                                           "per step (11 per ten-step run)"},
           "os_cpu_count": os.cpu_count(), "cpu_model": model}
    return out, {"x": x_ref, "v": v_ref, "ic32": ic32, "k": k_ref, "pk": p_ref}


def precision(lpc, synth, torch, oracle_small):
    """The GPU's ten-step run of the small configuration against the oracle's, from the same FP32 ICs."""
    import numpy as np
    w = synth.WORKLOADS["small"]
    ic = oracle_small["ic32"]
    dev = torch.device("cuda:0")
    ps = lpc.ParticleSet(*(torch.from_numpy(ic[k]).to(dev) for k in ("pos", "vel", "psi1", "psi2")),
                         id=torch.arange(w["n_side"] ** 3, dtype=torch.int32, device=dev))
    geom = lpc.geometry(w["n_side"], w["n_mesh"], w["box"])
    ws = lpc.workspace(geom, lpc.LPC_OP_COLA_STEP, dev)
    lpc.lpc_cola_step(geom, lpc.cosmology(**synth.COSMOLOGY), lpc.stepping(**synth.STEPPING), synth.A_LIST, ps, ws)
    x = ps.pos.cpu().numpy().astype(np.float64)
    v = ps.vel.cpu().numpy().astype(np.float64)
    box = w["box"]
    d = x - oracle_small["x"]
    d -= box * np.round(d / box)
    dv = v - oracle_small["v"]
    wsp = lpc.workspace(geom, lpc.LPC_OP_POWER_SPECTRUM, dev, n_particles=w["n_side"] ** 3)
    _, pk, cnt = lpc.lpc_power_spectrum(geom, ps.pos, 0.5, 20, wsp)
    sel = cnt > 0
    return {"workload": "32^3 particles, 64^3 mesh, 256 Mpc/h, seed 1, ten modified-COLA steps from the same FP32 "
                        "ICs; P(k) in 20 bins to k = 0.5 h/Mpc on the 64^3 mesh",
            "pos_max_abs_over_L": float(np.abs(d).max() / box), "pos_rms_over_L": float(np.sqrt(np.mean(d**2)) / box),
            "vel_rms_rel": float(np.sqrt(np.mean(dv**2)) / np.sqrt(np.mean(oracle_small["v"] ** 2))),
            "pk_max_rel": float(np.abs(pk[sel] / oracle_small["pk"][sel] - 1.0).max())}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="single", choices=["single", "small", "large"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline and the precision object")
    ap.add_argument("--no-batched", action="store_true", help="skip the 48-box batched measurement")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-correction measurement")
    ap.add_argument("--no-large", action="store_true", help="skip the large single-box measurement")
    ap.add_argument("--no-lightcone", action="store_true", help="skip the lightcone measurement")
    ap.add_argument("--no-tune", action="store_true", help="keep the built-in FFT tile widths (no autotuning)")
    ap.add_argument("--tiling-cache", default=None,
                    help="JSON cache of tuned FFT tile widths: applied if present, written with new results")
    ap.add_argument("--calib-copy", action="store_true",
                    help="first run one 1 GiB device-to-device copy (a known-size kernel for HBM counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the path has no multi-GPU form (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.steps < 1:
        print("--steps must be at least 1", file=sys.stderr)
        sys.exit(2)

    import synth
    # the CPU baseline first: its worker processes fork a process that has not touched the GPU
    cpu, oracle_small = None, None
    if not args.no_cpu:
        note("cpu baseline (FP64 oracle on the host)")
        cpu, oracle_small = cpu_baseline(workers=min(os.cpu_count() or 1, 16))

    import torch

    from paper_1506_03737_amd import autotune, lpc

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    w = synth.WORKLOADS[args.workload]
    n_side, nm, box = w["n_side"], w["n_mesh"], w["box"]
    tune_sizes = [nm]
    if not args.no_batched and args.workload == "single":
        tune_sizes += sorted({b["n_mesh"] for b in synth.batch_workload()})
    t_tune = time.perf_counter()
    if not args.no_tune:
        autotune.tune_sizes(tune_sizes, "cuda", path=args.tiling_cache,
                            log=lambda m: print(m, file=sys.stderr, flush=True))
    t_tune = time.perf_counter() - t_tune
    tilings = {str(s): lpc.lpc_fft_tiling_get(s) for s in tune_sizes}
    n = n_side**3
    dev = torch.device("cuda:0")
    geom = lpc.geometry(n_side, nm, box)
    cosmo = lpc.cosmology(**synth.COSMOLOGY)
    step = lpc.stepping(**synth.STEPPING)

    if args.calib_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    copy_gbs = copy_peak(torch)

    ic = make_ic(lpc, torch, n_side, box, w["seed"], cosmo)
    ps = lpc.ParticleSet.empty(n, dev)
    ws = lpc.workspace(geom, lpc.LPC_OP_COLA_STEP, dev)

    def reset():
        for k in ("pos", "vel", "psi1", "psi2", "id"):
            getattr(ps, k).copy_(getattr(ic, k))

    if args.warmup > 0:
        timed_schedule(lpc, torch, geom, cosmo, step, synth.A_LIST, ps, ws, reset, args.warmup, False)
    note(f"single box: {args.steps} timed steps")
    dt, stats = timed_schedule(lpc, torch, geom, cosmo, step, synth.A_LIST, ps, ws, reset, args.steps, True)
    note(f"single box: {dt * 1e3 / args.steps:.2f} ms per step")

    value = n * args.steps / dt
    evals = sum(m + 1 for m in schedule_runs(args.steps))
    stages = stage_table(stats, n, nm, dt * 1e3, evals, copy_gbs)
    dom = max((k for k in stats if stage_bytes(k, n, nm) is not None), key=lambda k: stats[k][1])
    dl, dms = stats[dom]
    share = launch_share(dom, dl, evals)
    dbytes = stage_bytes(dom, n, nm) * share  # per launch
    achieved = dbytes / (dms / dl * 1e-3) / 1e9
    width = next((tilings[str(nm)][f] for f, (st, _) in autotune.FIELDS.items() if dom in st), None)
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": MEASURED_TRAFFIC.get((dom, nm, width)),
                "algorithmic_bytes_per_launch": round(dbytes), "moved_bytes_per_launch": round(moved_bytes(dom, n, nm) * share),
                "tile_width": width, "launches": dl, "launches_per_evaluation": round(dl / evals, 3),
                "mean_launch_ms": round(dms / dl, 4), "copy_peak": round(copy_gbs, 1),
                "frac_of_copy": round(achieved / copy_gbs, 4)}

    out = {
        "metric": METRIC, "value": value, "unit": "particle-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt * 1e3 / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{args.workload}: {n_side}^3 particles, {nm}^3 mesh, {box:g} Mpc/h, 2LPT ICs at z=9, "
                               f"ten modified-COLA steps nLPT=-2.5, plain form", "n_side": n_side, "n_mesh": nm,
                   "box": box, "form": "plain", "schedule_calls": schedule_runs(args.steps),
                   "force_evaluations": sum(m + 1 for m in schedule_runs(args.steps)), "fft_tiling": tilings,
                   "fft_tiling_source": "built-in" if args.no_tune else "autotuned", "autotune_s": round(t_tune, 2)},
        "roofline": roofline,
        "stages": stages,
    }
    if not args.no_lightcone and args.workload == "single":
        note("lightcone")
        out["lightcone"] = lightcone_bench(lpc, synth, torch, ic, geom, ws, n)
    del ps, ws, ic
    torch.cuda.empty_cache()
    if not args.no_batched and args.workload == "single":
        note("batched (48 boxes)")
        out["batched"] = batched_bench(lpc, synth, torch)
        torch.cuda.empty_cache()
    if not args.no_learned and args.workload == "single":
        note("learned (pairs, training, calibration, runs)")
        out["learned"] = learned_bench(lpc, synth, torch)
        torch.cuda.empty_cache()
    if not args.no_large and args.workload == "single":
        note("large box")
        out["large"] = large_bench(lpc, synth, torch, copy_gbs)
    if cpu is not None:
        out["cpu_baseline"] = cpu
        note("precision")
        out["precision"] = precision(lpc, synth, torch, oracle_small)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
