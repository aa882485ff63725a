"""FFT tile autotuner for liblpc (lpc_fft_tiling_* in include/lpc.h).

Each FFT pass of the force path stages a tile of independent 1-D transforms through LDS; the tile width trades LDS
footprint (workgroups per CU) against loads in flight per workgroup, and the best width depends on the mesh size.
`tune` measures, for one mesh size, every instantiated width that fits, with the per-stage HIP-event timer of the
library on a PM force evaluation of uniform random particles, and keeps the fastest width per pass. Results are
kept in a JSON cache keyed by the GPU's architecture name and the mesh size, and `apply` hands them back to the
library. The widths change only the schedule, never the arithmetic of a column, so forces are identical under any
tiling.
"""
import json
import os
import time

from paper_1506_03737_amd import lpc

# Tiling field -> (the force-path stages it shapes, the instantiated widths)
FIELDS = {
    "z_rows": (("fft z r2c",), (8, 16, 32)),
    "axis_cols": (("fft y", "fft y inv"), (8, 16, 32)),
    "poisson_cols": (("fft x + poisson",), (4, 8, 16)),
    "c2r_rows": (("fft z c2r",), (4, 8, 16)),
}


def candidates(n_mesh):
    """{field: widths that fit n_mesh}, each checked by the library with the other fields at their defaults."""
    base = lpc.lpc_fft_tiling_default(n_mesh)
    saved = lpc.lpc_fft_tiling_get(n_mesh)
    out = {}
    try:
        for field, (_, widths) in FIELDS.items():
            ok = []
            for w in widths:
                t = dict(base, **{field: w})
                try:
                    lpc.lpc_fft_tiling_set(n_mesh, t)
                    ok.append(w)
                except lpc.LpcError:
                    pass
            out[field] = ok
    finally:
        lpc.lpc_fft_tiling_set(n_mesh, None if saved == base else saved)
    return out


def _stage_ms(run, reps):
    lpc.lpc_profile_reset()
    lpc.lpc_profile_enable(True)
    try:
        for _ in range(reps):
            run()
    finally:
        lpc.lpc_profile_enable(False)
    stats = lpc.lpc_profile_stats()
    lpc.lpc_profile_reset()
    return {k: ms / max(1, n) for k, (n, ms) in stats.items()}


TIE = 0.03  # widths timed within 3 % of the fastest count as tied


def pick(times, tie=TIE):
    """The width to use from {width: ms}: the widest one within `tie` of the fastest. Widths that close are within
    the timing noise of one tuning round, and the wider tile is kept because a batched launch runs every box at the
    narrowest width any of its mesh sizes was given."""
    fastest = min(times.values())
    return max(w for w, t in times.items() if t <= fastest * (1.0 + tie))


def tune(n_mesh, device="cuda", reps=5, box=1000.0, seed=0, log=None):
    """Measure every fitting width of every pass at mesh size n_mesh and set the fastest (see pick) as the override.

    The passes are separate kernels, so round i runs every field at its i-th candidate (the last one repeated when a
    field has fewer) and each field is ranked by its own stages' times: max(len(candidates)) rounds in all.
    Returns {"n_mesh", "tiling", "default", "stage_ms": {field: {width: ms}}, "seconds"}."""
    import torch
    t0 = time.perf_counter()
    cands = candidates(n_mesh)
    base = lpc.lpc_fft_tiling_default(n_mesh)
    n_part = max(1, n_mesh // 4) ** 3
    gen = torch.Generator(device="cpu").manual_seed(seed)
    pos = (torch.rand((3, n_part), generator=gen, dtype=torch.float64) * box).float().to(device)
    grad = torch.empty((3, n_part), dtype=torch.float32, device=device)
    geom = lpc.geometry(0, n_mesh, box)
    step = lpc.stepping()
    ws = lpc.workspace(geom, lpc.LPC_OP_PM_FORCE, device, n_particles=n_part)

    def run():
        lpc.lpc_pm_force(geom, step, pos, grad, ws)

    timings = {f: {} for f in FIELDS}
    saved = lpc.lpc_fft_tiling_get(n_mesh)
    try:
        for i in range(max(len(c) for c in cands.values())):
            t = {f: cands[f][min(i, len(cands[f]) - 1)] for f in FIELDS}
            lpc.lpc_fft_tiling_set(n_mesh, t)
            run()  # warm-up under this tiling
            torch.cuda.synchronize()
            ms = _stage_ms(run, reps)
            for f, (stages, _) in FIELDS.items():
                timings[f].setdefault(t[f], sum(ms[s] for s in stages))
    except BaseException:
        lpc.lpc_fft_tiling_set(n_mesh, None if saved == base else saved)
        raise
    best = {f: pick(timings[f]) for f in FIELDS}
    lpc.lpc_fft_tiling_set(n_mesh, best)
    res = {"n_mesh": n_mesh, "tiling": best, "default": base,
           "stage_ms": {f: {str(w): round(v, 4) for w, v in timings[f].items()} for f in FIELDS},
           "seconds": time.perf_counter() - t0}
    if log:
        log(f"fft tiling {n_mesh}: {best} (default {base}); stage ms {res['stage_ms']}")
    return res


def arch_name(device=0):
    import torch
    return str(torch.cuda.get_device_properties(device).gcnArchName).split(":")[0]


def load(path):
    """The cache file as {arch: {mesh size (str): tiling}}, empty if the file does not exist."""
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def save(path, results, arch):
    """Merge tuned results (from `tune`) into the cache file under `arch`."""
    cache = load(path)
    entry = cache.setdefault(arch, {})
    for r in results:
        entry[str(r["n_mesh"])] = r["tiling"]
    d = os.path.dirname(os.path.abspath(path))
    os.makedirs(d, exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def apply(path, arch):
    """Set the cached tilings of `arch` as overrides; returns the mesh sizes set. An entry the library rejects (a
    cache from another build) is skipped."""
    done = []
    for n, t in load(path).get(arch, {}).items():
        try:
            lpc.lpc_fft_tiling_set(int(n), t)
            done.append(int(n))
        except (lpc.LpcError, KeyError, TypeError, ValueError):
            pass
    return sorted(done)


def tune_sizes(sizes, device="cuda", path=None, reps=5, log=None):
    """Tune every mesh size in `sizes` (skipping those already in the cache at `path`, which are applied instead);
    returns the new results. With a path, the results are merged into the cache."""
    arch = arch_name()
    cached = set(apply(path, arch)) if path else set()
    results = [tune(n, device, reps=reps, log=log) for n in sizes if n not in cached]
    if path and results:
        save(path, results, arch)
    return results
