"""Training and use of the learned displacement correction (the network of include/lpc.h), on top of the C ABI.

A pair is two runs of lpc_cola_step from the same 2LPT initial conditions: a coarse one with the PM mesh equal to the
particle lattice (Nm = N) and a fine one with Nm = 3 N. The network learns the per-particle displacement that moves
the coarse result onto the fine one (in lattice units, as a field on the N^3 lattice), so that a coarse run plus one
network pass stands in for the fine run. Every numerical step runs in liblpc's kernels; this module only sequences
calls and holds device buffers (torch tensors).
"""
import time

import numpy as np

from paper_1506_03737_amd import lpc


def run_pair(seed, n_side, box, a_list, cosmo, step, device, fine_factor=3):
    """(coarse, fine) particle sets evolved over a_list from the same initial conditions (lattice-ordered ids)."""
    import torch
    n = n_side**3
    geom_ic = lpc.geometry(n_side, n_side, box)
    ic = lpc.ParticleSet.empty(n, device)
    ws = lpc.workspace(geom_ic, lpc.LPC_OP_INIT_IC, device)
    lpc.lpc_init_ic(geom_ic, cosmo, seed, a_list[0], ic, ws)
    del ws
    out = []
    for nm in (n_side, fine_factor * n_side):
        ps = lpc.ParticleSet(*(torch.clone(getattr(ic, k)) for k in ("pos", "vel", "psi1", "psi2", "id")))
        geom = lpc.geometry(n_side, nm, box)
        ws = lpc.workspace(geom, lpc.LPC_OP_COLA_STEP, device)
        lpc.lpc_cola_step(geom, cosmo, step, a_list, ps, ws)
        del ws
        out.append(ps)
    return out[0], out[1]


def pair_grids(coarse, fine, n_side, box, ws, device):
    """Input grid (coarse displacement from the lattice and Psi1, FP32 [N^3][6]) and target grid (fine - coarse,
    FP32 [N^3][3])."""
    import torch
    geom = lpc.geometry(n_side, n_side, box)
    feat = torch.empty((n_side**3, lpc.NET_INPUT_CHANNELS), dtype=torch.float32, device=device)
    target = torch.empty((n_side**3, 3), dtype=torch.float32, device=device)
    lpc.lpc_net_features(geom, coarse.pos, coarse.id, feat, ws, psi1=coarse.psi1)
    lpc.lpc_net_features(geom, fine.pos, fine.id, target, ws, ref_pos=coarse.pos)
    return feat, target


def symmetry(grid, n_side, k):
    """The k-th (0..47) symmetry of the cube applied to a field of 3-vectors [N^3][3 m] (m vectors per site): an axis
    permutation with reflections, acting on both the grid positions and every vector's components (the equations of
    motion are invariant under it). Runs in liblpc (lpc_net_symmetry)."""
    return lpc.lpc_net_symmetry(n_side, k, grid)


def train(samples, n_side, epochs, lr, seed=1, device="cuda", augment=True, lr_final=None, log=None):
    """Adam on (feature, target) grid pairs, with the learning rate decaying from lr to lr_final (cosine) when
    lr_final is given; returns (params on device, per-epoch mean losses)."""
    import torch
    params = torch.from_numpy(lpc.lpc_net_init(seed)).to(device)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    grad = torch.empty_like(params)
    ws = lpc.net_workspace(n_side, device)
    rng = np.random.default_rng(seed)
    t = 0
    history = []
    for ep in range(epochs):
        order = rng.permutation(len(samples))
        losses = []
        for i in order:
            feat, target = samples[i]
            if augment:
                k = int(rng.integers(48))
                feat, target = symmetry(feat, n_side, k), symmetry(target, n_side, k)
            t += 1
            rate = lr
            if lr_final is not None:
                frac = (t - 1) / max(1, epochs * len(samples) - 1)
                rate = lr_final + 0.5 * (lr - lr_final) * (1.0 + np.cos(np.pi * frac))
            losses.append(lpc.lpc_net_loss_grad(n_side, params, feat, target, grad, ws))
            lpc.lpc_net_adam(params, m, v, grad, t, rate)
        history.append(float(np.mean(losses)))
        if log:
            log(f"epoch {ep}: mean loss {history[-1]:.4e}")
    return params, history


def validation_loss(params, samples, n_side, device="cuda"):
    """Mean loss of the network and of the zero correction (mean target^2) over held-out samples. The zero
    correction's loss is the library's loss at all-zero parameters: every layer's output is then exactly zero."""
    import torch
    ws = lpc.net_workspace(n_side, device)
    grad = torch.empty_like(params)
    zeros = torch.zeros_like(params)
    net, zero = [], []
    for feat, target in samples:
        net.append(lpc.lpc_net_loss_grad(n_side, params, feat, target, grad, ws))
        zero.append(lpc.lpc_net_loss_grad(n_side, zeros, feat, target, grad, ws))
    return float(np.mean(net)), float(np.mean(zero))


def power_spectrum(pos, n, box, device, nm_est=512, k_max=1.0, n_bins=100):
    """Binned P(k) of particles on an nm_est^3 estimator mesh (lpc_power_spectrum)."""
    g = lpc.geometry(0, nm_est, box)
    ws = lpc.workspace(g, lpc.LPC_OP_POWER_SPECTRUM, device, n_particles=n)
    return lpc.lpc_power_spectrum(g, pos, k_max, n_bins, ws)


def pk_max_error(pos, ref_pos, n, box, device, k_eval=0.5, nm_est=512, n_bins=100):
    """max over k <= k_eval of |P(pos) / P(ref_pos) - 1| (binned P(k), empty bins skipped)."""
    k, p_ref, cnt = power_spectrum(ref_pos, n, box, device, nm_est=nm_est, n_bins=n_bins)
    _, p, _ = power_spectrum(pos, n, box, device, nm_est=nm_est, n_bins=n_bins)
    sel = (k <= k_eval) & (cnt > 0)
    return float(np.max(np.abs(p[sel] / p_ref[sel] - 1.0)))


def corrected(params, coarse, n_side, box, device, ws=None):
    """A copy of a coarse run's particles moved by the network (lpc_net_apply)."""
    import torch
    out = lpc.ParticleSet(torch.clone(coarse.pos), None, coarse.psi1, None, coarse.id)
    lpc.lpc_net_apply(lpc.geometry(n_side, n_side, box), params, out, ws if ws is not None else lpc.net_workspace(n_side, device))
    return out


# Output gains tried by calibrate_gain
GAINS = tuple(round(0.40 + 0.05 * i, 2) for i in range(13))


def calibrate_gain(params, runs, n_side, box, device, gains=GAINS, nm_est=None, n_bins=50, k_eval=0.5):
    """The output gain that makes the corrected held-out runs' P(k) match their fine runs' best.

    A network trained on the mean squared displacement error returns, at each site, the mean residual given its
    inputs; moved by it, particles cluster more than the fine run's at k ~ 0.3-0.5 h/Mpc. One scalar on the output
    layer (lpc_net_scale_output) trades that back: for every g in gains the held-out coarse runs are corrected with
    g network(x) and scored by the mean over runs of max_{k <= k_eval} |P_corr / P_fine - 1|. runs: [(coarse, fine)]
    particle sets that were not trained on. Returns (best g, params scaled by it (a copy), {g: error})."""
    import torch
    nm_est = nm_est or 2 * n_side
    ws = lpc.net_workspace(n_side, device)
    errors = {}
    for g in gains:
        pg = torch.clone(params)
        lpc.lpc_net_scale_output(pg, g)
        errs = [pk_max_error(corrected(pg, c, n_side, box, device, ws).pos, f.pos, n_side**3, box, device,
                             k_eval, nm_est, n_bins) for c, f in runs]
        errors[g] = float(np.mean(errs))
    best = min(errors, key=errors.get)
    pb = torch.clone(params)
    lpc.lpc_net_scale_output(pb, best)
    return best, pb, errors


def fit_correction(train_seeds, val_seeds, n_side, box, a_list, cosmo, step, device, epochs, lr=1e-3, lr_final=5e-5,
                   seed=3, log=None):
    """The whole recipe: coarse/fine pairs of the train and held-out seeds, Adam over the training pairs with random
    cube symmetries, the held-out loss against no correction, then the output gain calibrated on the held-out runs.
    Returns a dict: params (gain applied), gain, gain_errors, history, validation_loss_ratio (before the gain),
    pairs_s, train_s, calibrate_s."""
    import torch
    ws = lpc.net_workspace(n_side, device)
    t0 = time.perf_counter()
    train_s = []
    for sd in train_seeds:
        c, f = run_pair(sd, n_side, box, a_list, cosmo, step, device)
        train_s.append(pair_grids(c, f, n_side, box, ws, device))
        del c, f
    val_runs = [run_pair(sd, n_side, box, a_list, cosmo, step, device) for sd in val_seeds]
    val_s = [pair_grids(c, f, n_side, box, ws, device) for c, f in val_runs]
    torch.cuda.synchronize()
    t_pairs = time.perf_counter() - t0
    (params, hist), t_train = timed(lambda: train(train_s, n_side, epochs=epochs, lr=lr, lr_final=lr_final, seed=seed,
                                                  device=device, log=log))
    del train_s
    net_loss, zero_loss = validation_loss(params, val_s, n_side, device)
    (gain, scaled, errors), t_cal = timed(lambda: calibrate_gain(params, val_runs, n_side, box, device))
    if log:
        log(f"held-out loss ratio {net_loss / zero_loss:.4f}; gain {gain} (held-out P(k) errors {errors})")
    return {"params": scaled, "gain": gain, "gain_errors": errors, "history": hist,
            "validation_loss_ratio": net_loss / zero_loss, "pairs_s": t_pairs, "train_s": t_train,
            "calibrate_s": t_cal}


def timed(fn):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = fn()
    torch.cuda.synchronize()
    return out, time.perf_counter() - t0
