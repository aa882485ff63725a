"""Throughput benchmark of the PM-COLA time step on one MI355X.

Workload (the single-box configuration): 256^3 particles, 768^3 mesh, 1000 Mpc/h box, 2LPT initial conditions at
z = 9 from a seeded BBKS Gaussian field (generated on the GPU by lpc_init_ic, untimed), modified COLA stepping with
nLPT = -2.5, CIC window deconvolved once.

A "step" is one COLA time step: drift + full PM force (deposit, r2c FFT, Poisson/gradient, 3 c2r, gather) + kick.
The timed region is ONE lpc_cola_step call over K + 1 scale factors spaced uniformly from a = 0.1 to 1.0: the opening
force and half kick, K drift/force/kick iterations and the frame-velocity conversions (K + 1 force evaluations in
all). value = N^3 * K / wall time (particle-steps/s), inputs resident in HBM before the clock starts.

Also reported: the dominant kernel's achieved HBM bandwidth from HIP events recorded on the call's stream
(roofline), the FP64 CPU oracle's rate on a bounded sample (cpu_baseline), and the batched form on 48 uneven boxes
(96^3/128^3/160^3 particles, Nm = 2N, L = 300..600 Mpc/h, one lpc_cola_step_batched call replaying its recorded HIP
graph; aggregate particle-steps/s, in "batched"), and the learned form (a coarse Nm = N run plus the trained
correction network against the fine Nm = 3N run, with its P(k) error, in "learned").

Before the clock starts, the FFT tile widths of every mesh size measured here are autotuned (paper_1506_03737_amd/
autotune.py; --no-tune keeps the built-in widths); the widths used are reported in config.fft_tiling.

Usage: python bench.py [--gpus 1] [--steps 10] [--warmup 1] [--workload single|small|large] [--no-cpu] [--no-batched]
                      [--no-learned] [--no-tune] [--tiling-cache PATH]
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

# HBM bytes per launch measured with rocprofv3 FETCH_SIZE / WRITE_SIZE passes (read scaled by 2.0, write by 1.0, from
# a 1 GiB copy), by (stage, mesh size, tile width of the stage); profiles/force_path_768_hbm_traffic.md. Must be
# re-measured (or removed) when the kernel changes.
MEASURED_TRAFFIC = {("fft z c2r", 768, 4): 10.985e9, ("fft y inv", 768, 8): 9.255e9, ("fft x + poisson", 768, 8): 5.664e9,
                    ("fft y", 768, 8): 3.713e9, ("fft z r2c", 768, 16): 3.643e9}


def stage_bytes(stage, n_part, nm, ncomp_y=3):
    """Algorithmic HBM bytes of one launch of each force-path stage (FP32 mesh, int64 density, SoA particles).

    Half spectra are counted at nm * nm * (nm/2 + 1) complex values (8 B each)."""
    M = nm**3
    H = nm * nm * (nm // 2 + 1) * 8        # bytes of one half-spectrum complex mesh
    corners = min(M, 8 * n_part)
    return {
        "deposit": 12 * n_part + 4 * M,     # read positions, the FP32 density contrast written once
        "fft z r2c": 4 * M + H,             # read the FP32 contrast, write half spectrum
        "fft y": 2 * H,
        "fft x + poisson": H + 2 * H,       # read delta_hat, write the x gradient and the potential
        "fft y inv": 2 * H + 3 * H,         # x gradient in place; read the potential, write its y gradient and itself
        "fft z c2r": 3 * H + 12 * M,        # read three spectra, write the AoS float3 force mesh
        # pos, vel, psi1, psi2 in, vel and pos out, the next sort's key and rank out (on the launches that drift)
        "gather kick drift": 80 * n_part + 12 * corners,
        "frame velocity": 48 * n_part,      # read vel, psi1, psi2; write vel
    }.get(stage)


def stage_table(stats, n_part, nm, wall_ms):
    stages = {}
    for name, (launches, ms) in stats.items():
        b = stage_bytes(name, n_part, nm)
        avg = ms / launches
        entry = {"launches": launches, "avg_ms": round(avg, 4), "share": round(ms / wall_ms, 4)}
        if b is not None:
            entry["GB_per_s"] = round(b / (avg * 1e-3) / 1e9, 1)
        stages[name] = entry
    return stages


def batched_bench(lpc, synth, torch, steps):
    """The 48-box batched form: ICs per box (untimed), one recording call, then one timed replay of the graph over
    steps + 1 scale factors. Returns the "batched" object of the JSON line."""
    import numpy as np
    dev = torch.device("cuda:0")
    cosmo = lpc.cosmology(**synth.COSMOLOGY)
    step = lpc.stepping(**synth.STEPPING)
    boxes = synth.batch_workload()
    ics, sets, entries = [], [], []
    for b in boxes:
        n = b["n_side"] ** 3
        geom = lpc.geometry(b["n_side"], b["n_mesh"], b["box"])
        ic = lpc.ParticleSet.empty(n, dev)
        ws_ic = lpc.workspace(geom, lpc.LPC_OP_INIT_IC, dev)
        lpc.lpc_init_ic(geom, cosmo, b["seed"], 0.1, ic, ws_ic)
        del ws_ic
        ps = lpc.ParticleSet.empty(n, dev)
        ics.append(ic)
        sets.append(ps)
        entries.append((geom, ps))
    ws = lpc.workspace_batched(entries, dev)
    n_total = sum(b["n_side"] ** 3 for b in boxes)

    def reset():
        for ps, ic in zip(sets, ics):
            for k in ("pos", "vel", "psi1", "psi2", "id"):
                getattr(ps, k).copy_(getattr(ic, k))

    a_list = np.linspace(0.1, 1.0, steps + 1)
    reset()
    lpc.lpc_cola_step_batched(entries, cosmo, step, a_list, ws)  # records the graph (untimed)
    reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lpc.lpc_cola_step_batched(entries, cosmo, step, a_list, ws)  # replays it
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # per-stage times from one more (direct-launch, event-bracketed) run
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
    # algorithmic bytes of a batched launch: the sum over boxes of each box's bytes
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
                        "2LPT ICs at z=9, modified COLA nLPT=-2.5; one graph replay (graph recorded by an untimed "
                        "identical call)",
            "stages_direct_launch": stages}


def learned_bench(lpc, synth, torch, steps):
    """The learned form: a coarse run (Nm = N) plus one network pass, against the fine run (Nm = 3N) it stands in
    for. Training data: 64 coarse/fine pairs of 128^3 particles in 500 Mpc/h boxes (seeds 5000..5063) made by
    lpc_cola_step, 8 more held out; 12 epochs of Adam (lr 1e-3 -> 5e-5, cosine), random cube symmetries. Applied to
    the single-box workload (256^3 particles, 1000 Mpc/h, seed 2015): coarse Nm = 256 + network vs fine Nm = 768.
    Throughput counts the coarse run and the network pass; P(k) errors are against the fine run, k <= 0.5 h/Mpc."""
    import numpy as np
    from paper_1506_03737_amd import learned
    dev = torch.device("cuda:0")
    cosmo = lpc.cosmology(**synth.COSMOLOGY)
    step = lpc.stepping(**synth.STEPPING)
    a_list = np.linspace(0.1, 1.0, steps + 1)
    n_tr, box_tr = 128, 500.0
    ws = lpc.net_workspace(n_tr, dev)
    t0 = time.perf_counter()
    train_s, val_s = [], []
    for seed in range(5000, 5072):
        c, f = learned.run_pair(seed, n_tr, box_tr, a_list, cosmo, step, dev)
        (train_s if seed < 5064 else val_s).append(learned.pair_grids(c, f, n_tr, box_tr, ws, dev))
        del c, f
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t0
    (params, hist), t_train = learned.timed(
        lambda: learned.train(train_s, n_tr, epochs=12, lr=1e-3, lr_final=5e-5, seed=3, device=dev))
    net_loss, zero_loss = learned.validation_loss(params, val_s, n_tr, dev)
    del train_s, val_s, ws
    # apply to the single-box workload
    N, box = 256, 1000.0
    n = N**3
    geom_ic = lpc.geometry(N, N, box)
    ic = lpc.ParticleSet.empty(n, dev)
    ws_ic = lpc.workspace(geom_ic, lpc.LPC_OP_INIT_IC, dev)
    lpc.lpc_init_ic(geom_ic, cosmo, 2015, 0.1, ic, ws_ic)
    del ws_ic
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
    k, p_fine, cnt = learned.power_spectrum(runs["fine"][0].pos, n, box, dev)
    _, p_coarse, _ = learned.power_spectrum(runs["coarse"][0].pos, n, box, dev)
    _, p_corr, _ = learned.power_spectrum(corrected.pos, n, box, dev)
    sel = (k <= 0.5) & (cnt > 0)
    err = lambda p: float(np.max(np.abs(p[sel] / p_fine[sel] - 1.0)))
    t_learned = runs["coarse"][1] + t_apply
    return {"value": n * steps / t_learned, "unit": "particle-steps/s", "ms_per_step": t_learned * 1e3 / steps,
            "fine_value": n * steps / runs["fine"][1], "speedup_vs_fine": runs["fine"][1] / t_learned,
            "coarse_run_ms": runs["coarse"][1] * 1e3, "net_apply_ms": t_apply * 1e3, "fine_run_ms": runs["fine"][1] * 1e3,
            "pk_max_rel_err_k_le_0.5": {"coarse": err(p_coarse), "coarse+net": err(p_corr)},
            "validation_loss_ratio": net_loss / zero_loss, "train_s": t_train, "pairs_s": t_gen,
            "workload": "256^3 particles, 1000 Mpc/h, seed 2015: coarse Nm=256 + network vs fine Nm=768; network "
                        "trained on 64 pairs of 128^3 / 500 Mpc/h (coarse Nm=128, fine Nm=384), 12 epochs"}


def cpu_baseline_sample():
    """The FP64 oracle, untuned, on two COLA steps of the single-box workload at 1/8 of its volume: 128^3 particles,
    384^3 mesh, 500 Mpc/h (same Nm/N = 3 and particle density). Returns particle-steps/s for that sample."""
    import numpy as np

    import synth
    from oracle import cola as ocola
    from oracle import ic as oic
    n_side, nm, box = 128, 384, 500.0
    init = oic.initial_conditions(7, n_side, box, 0.1, **synth.COSMOLOGY)
    t0 = time.perf_counter()
    ocola.cola_run(init["pos"], init["vel"], init["psi1"], init["psi2"], [0.1, 0.19, 0.28],
                   synth.COSMOLOGY["omega_m"], nm, box)
    dt = time.perf_counter() - t0
    # the run above is 2 drifts and 3 force evaluations (the GPU run: 10 drifts, 11 force evaluations)
    return {"value": 2 * n_side**3 / dt, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"two COLA steps (3 force evaluations + 2 drifts) of the FP64 NumPy oracle, 128^3 particles, "
                      f"384^3 mesh, 500 Mpc/h (single-box workload at 1/8 volume), {dt:.1f} s, single thread"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="single", choices=["single", "small", "large"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-batched", action="store_true", help="skip the 48-box batched measurement")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-correction measurement")
    ap.add_argument("--no-tune", action="store_true", help="keep the built-in FFT tile widths (no autotuning)")
    ap.add_argument("--tiling-cache", default=None,
                    help="JSON cache of tuned FFT tile widths: applied if present, written with new results")
    ap.add_argument("--calib-copy", action="store_true",
                    help="first run one 1 GiB device-to-device copy (a known-size kernel for HBM counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the path has no multi-GPU form (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_1506_03737_amd import autotune, lpc

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    w = synth.WORKLOADS[args.workload]
    n_side, nm, box = w["n_side"], w["n_mesh"], w["box"]
    # FFT tile widths: tuned (untimed) for the single-box mesh and the batched form's meshes
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

    ic = lpc.ParticleSet.empty(n, dev)
    ws_ic = lpc.workspace(geom, lpc.LPC_OP_INIT_IC, dev)
    lpc.lpc_init_ic(geom, cosmo, w["seed"], 0.1, ic, ws_ic)
    del ws_ic
    ps = lpc.ParticleSet.empty(n, dev)
    ws = lpc.workspace(geom, lpc.LPC_OP_COLA_STEP, dev)

    def reset():
        for k in ("pos", "vel", "psi1", "psi2", "id"):
            getattr(ps, k).copy_(getattr(ic, k))

    if args.warmup > 0:
        reset()
        lpc.lpc_cola_step(geom, cosmo, step, np.linspace(0.1, 1.0, args.warmup + 1), ps, ws)
    reset()
    a_list = np.linspace(0.1, 1.0, args.steps + 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lpc.lpc_cola_step(geom, cosmo, step, a_list, ps, ws)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # the same run again with per-stage HIP events (they add a record between launches, so they stay out of the
    # timed run above)
    reset()
    lpc.lpc_profile_reset()
    lpc.lpc_profile_enable(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lpc.lpc_cola_step(geom, cosmo, step, a_list, ps, ws)
    torch.cuda.synchronize()
    dt_prof = time.perf_counter() - t1
    lpc.lpc_profile_enable(False)
    stats = lpc.lpc_profile_stats()

    value = n * args.steps / dt
    stages = stage_table(stats, n, nm, dt_prof * 1e3)
    dom = max((k for k in stats if stage_bytes(k, n, nm) is not None), key=lambda k: stats[k][1])
    dl, dms = stats[dom]
    dbytes = stage_bytes(dom, n, nm)
    achieved = dbytes / (dms / dl * 1e-3) / 1e9
    width = next((tilings[str(nm)][f] for f, (st, _) in autotune.FIELDS.items() if dom in st), None)
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": MEASURED_TRAFFIC.get((dom, nm, width)),
                "algorithmic_bytes_per_launch": dbytes, "tile_width": width}

    out = {
        "metric": METRIC, "value": value, "unit": "particle-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt * 1e3 / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{args.workload}: {n_side}^3 particles, {nm}^3 mesh, {box:g} Mpc/h, 2LPT ICs at z=9, "
                               f"modified COLA nLPT=-2.5, plain form", "n_side": n_side, "n_mesh": nm, "box": box,
                   "form": "plain", "force_evaluations": args.steps + 1, "fft_tiling": tilings,
                   "fft_tiling_source": "built-in" if args.no_tune else "autotuned",
                   "autotune_s": round(t_tune, 2)},
        "roofline": roofline,
        "stages": stages,
    }
    if not args.no_batched and args.workload == "single":
        del ps, ic, ws
        torch.cuda.empty_cache()
        out["batched"] = batched_bench(lpc, synth, torch, args.steps)
    if not args.no_learned and args.workload == "single":
        torch.cuda.empty_cache()
        out["learned"] = learned_bench(lpc, synth, torch, args.steps)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline_sample()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
