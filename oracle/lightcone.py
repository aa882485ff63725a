"""On-the-fly lightcone with box replicates, in float64.

Oracle (test infrastructure only). Follows Sec. 6.1 of Howlett, Manera & Percival (2015): the COLA run of Sec. 2.3
with a modified drift. In every drift a_i -> a_{i+1} of the lightcone, a particle image is output when it leaves the
shrinking lightcone, i.e. when its comoving distance R_p from the observer satisfies R_p,i <= R_L,i and
R_p,i+1 > R_L,i+1, with R_L(a) the comoving distance to scale factor a. The crossing time a_L comes from the linear
interpolation of R_p and R_L between a_i and a_{i+1} (the interpolation equation of Sec. 6.1); the position is the
drift of Sec. 2.3 taken from a_i to a_L; the velocity is not interpolated (the momentum at a_{i+1/2}). Sec. 6.2 adds
replicates: the box is repeated on a lattice of offsets and every replicate's particles are tested the same way.
Sec. 6.1.1 measures the interpolation against the exact crossing; exact_crossing solves the crossing equation by
root finding for that check.

Readings taken (the paper leaves these open):
  * R_L(a) = (c / H0) int_a^1 da' / (a'^2 E(a')) with c / H0 = 2997.92458 Mpc/h (H0 = 100 h km/s/Mpc).
  * The lightcone is active on every drift whose start a_i is at or after a_start (the paper's first output time);
    the run itself starts at a_list[0].
  * A particle image is identified by the particle and the replicate offset o = L (i, j, k): its position at a_i is
    the wrapped position plus o, and its drifted position is x_i + o + dx with the unwrapped drift dx, so an image's
    path is continuous even where the particle wraps around the box during the drift.
  * The drift from a_i to a_L uses the step's own factors: the standard Q(a_i, a_L) = int da / (a^3 E), or the
    modified int u / (a^3 E) da / u(a_{i+1/2}) with u = a^nLPT (the same normalisation as the full drift), and
    D1(a_L) - D1(a_i), D2(a_L) - D2(a_i) for the 2LPT frame (COLA only).
  * The velocity output is the momentum p = a^2 dx/dt / H0 at a_{i+1/2}: the kicked residual momentum plus, for COLA,
    the frame momentum a^3 E (D1' Psi1 + D2' Psi2) evaluated at a_{i+1/2}.
  * a_L is clamped to [a_i, a_{i+1}] (the interpolated value can leave the interval only through rounding).
"""
import numpy as np
from scipy import integrate, optimize
from scipy.special import hyp2f1

from . import cosmology as cosmo
from .cola import kick_acceleration
from .pm import pm_force

C_OVER_H0 = 2997.92458  # Mpc/h


def comoving_distance(a, omega_m):
    """R_L(a) = (c / H0) int_a^1 da' / (a'^2 E(a')), Mpc/h (Sec. 6.1)."""
    f = lambda x: 1.0 / (x * x * float(cosmo.hubble_E(x, omega_m)))
    val, _ = integrate.quad(f, float(a), 1.0, epsabs=0.0, epsrel=1e-13, limit=200)
    return C_OVER_H0 * val


def partial_drift(a_i, a, a_ip1, omega_m, modified, n_lpt):
    """(Q, dD1, dD2) of the drift from a_i to a (a_i <= a <= a_{i+1}) within the step a_i -> a_{i+1} (Sec. 2.3)."""
    if modified:
        a_mid = 0.5 * (a_i + a_ip1)
        f = lambda x: x**n_lpt / (x**3 * float(cosmo.hubble_E(x, omega_m)))
        q = integrate.quad(f, a_i, a, epsabs=0.0, epsrel=1e-13, limit=200)[0] / a_mid**n_lpt
    else:
        f = lambda x: 1.0 / (x**3 * float(cosmo.hubble_E(x, omega_m)))
        q = integrate.quad(f, a_i, a, epsabs=0.0, epsrel=1e-13, limit=200)[0]
    dd1 = cosmo.growth_D1(a, omega_m) - cosmo.growth_D1(a_i, omega_m)
    dd2 = cosmo.growth_D2(a, omega_m) - cosmo.growth_D2(a_i, omega_m)
    return q, dd1, dd2


def growth_D1_many(a, omega_m):
    """D1 at many times at once: the flat-LCDM growing mode a 2F1(1/3, 1; 11/6; -a^3 OL / Om), normalised to
    D1(1) = 1 (the same function as cosmology.growth_D1, by an independent closed form)."""
    ol = 1.0 - omega_m
    f = lambda x: x * hyp2f1(1.0 / 3.0, 1.0, 11.0 / 6.0, -np.asarray(x, dtype=np.float64) ** 3 * ol / omega_m)
    return f(a) / f(1.0)


def growth_D2_many(a, omega_m):
    """Eq. 7 (Bouchet) at many times: -(3/7) D1^2 Om(a)^(-1/143)."""
    a = np.asarray(a, dtype=np.float64)
    return -3.0 / 7.0 * growth_D1_many(a, omega_m) ** 2 * cosmo.omega_m_of_a(a, omega_m) ** (-1.0 / 143.0)


def partial_drift_many(a_i, a, a_ip1, omega_m, modified, n_lpt):
    """partial_drift for an array of end times a: the drift integral by adaptive vector quadrature over
    t in [0, 1] with x = a_i + t (a - a_i), D1 and D2 by the closed form."""
    a = np.asarray(a, dtype=np.float64)
    span = a - a_i
    if modified:
        norm = (0.5 * (a_i + a_ip1)) ** n_lpt
        h = lambda x: x**n_lpt / (x**3 * cosmo.hubble_E(x, omega_m)) / norm
    else:
        h = lambda x: 1.0 / (x**3 * cosmo.hubble_E(x, omega_m))
    q = integrate.quad_vec(lambda t: span * h(a_i + t * span), 0.0, 1.0, epsabs=0.0, epsrel=1e-12)[0]
    dd1 = growth_D1_many(a, omega_m) - growth_D1_many(a_i, omega_m)
    dd2 = growth_D2_many(a, omega_m) - growth_D2_many(a_i, omega_m)
    return q, dd1, dd2


def replicate_offsets(box, rep_lo, rep_hi):
    """Offsets L (i, j, k) for i in [lo_x, hi_x], ... (x slowest), shape (R, 3), and their flat indices."""
    axes = [np.arange(lo, hi + 1) for lo, hi in zip(rep_lo, rep_hi)]
    I, J, K = np.meshgrid(*axes, indexing="ij")
    offs = box * np.stack([I.ravel(), J.ravel(), K.ravel()], axis=1).astype(np.float64)
    return offs, np.arange(offs.shape[0])


def drift_crossings(x_i, p, psi1, psi2, a_i, a_ip1, omega_m, box, origin, rep_lo, rep_hi, cola, modified, n_lpt,
                    index=None):
    """Particle images that leave the lightcone during the drift a_i -> a_{i+1} (Sec. 6.1).

    x_i: wrapped positions at a_i (3, n); p: residual momentum after the kick at a_i (the momentum at a_{i+1/2});
    psi1, psi2: 2LPT displacements. Returns a dict of arrays over the crossings: index, replicate, a (a_L), pos (3, m),
    vel (3, m)."""
    n = x_i.shape[1]
    index = np.arange(n) if index is None else np.asarray(index)
    q, dd1, dd2 = partial_drift(a_i, a_ip1, a_ip1, omega_m, modified, n_lpt)
    dx = q * p
    if cola:
        dx = dx + dd1 * psi1 + dd2 * psi2
    r_li = comoving_distance(a_i, omega_m)
    r_ln = comoving_distance(a_ip1, omega_m)
    a_mid = 0.5 * (a_i + a_ip1)
    v = np.array(p, dtype=np.float64)
    if cola:
        f1, f2 = cosmo.frame_momentum_factors(a_mid, omega_m)
        v = v + f1 * psi1 + f2 * psi2
    o = np.asarray(origin, dtype=np.float64)[:, None]
    offs, rep_ids = replicate_offsets(box, rep_lo, rep_hi)
    parts = []
    for off, rid in zip(offs, rep_ids):
        start = x_i + off[:, None]
        r_pi = np.sqrt(np.sum((start - o) ** 2, axis=0))
        r_pn = np.sqrt(np.sum((start + dx - o) ** 2, axis=0))
        hit = np.flatnonzero((r_pi <= r_li) & (r_pn > r_ln))
        if hit.size:
            parts.append((hit, np.full(hit.size, rid), off, r_pi[hit], r_pn[hit]))
    if not parts:
        return {"index": np.zeros(0, np.int64), "replicate": np.zeros(0, np.int64), "a": np.zeros(0),
                "pos": np.zeros((3, 0)), "vel": np.zeros((3, 0))}
    k = np.concatenate([h for h, _, _, _, _ in parts])
    rid = np.concatenate([r for _, r, _, _, _ in parts])
    off = np.concatenate([np.repeat(f[:, None], h.size, axis=1) for h, _, f, _, _ in parts], axis=1)
    r_pi = np.concatenate([a for _, _, _, a, _ in parts])
    r_pn = np.concatenate([b for _, _, _, _, b in parts])
    # Sec. 6.1: R_p and R_L both interpolated linearly in a between a_i and a_{i+1}
    a_l = a_i + (a_ip1 - a_i) * (r_li - r_pi) / ((r_pn - r_pi) - (r_ln - r_li))
    a_l = np.clip(a_l, a_i, a_ip1)
    ql, d1l, d2l = partial_drift_many(a_i, a_l, a_ip1, omega_m, modified, n_lpt)
    xl = x_i[:, k] + off + ql * p[:, k]
    if cola:
        xl = xl + d1l * psi1[:, k] + d2l * psi2[:, k]
    return {"index": index[k].astype(np.int64), "replicate": rid.astype(np.int64), "a": a_l, "pos": xl,
            "vel": v[:, k]}


def exact_crossing(x_i, p, psi1, psi2, a_i, a_ip1, omega_m, origin, cola, modified, n_lpt):
    """The exact crossing time of one particle image (Sec. 6.1.1): the root in [a_i, a_{i+1}] of
    |x(a) - origin| = R_L(a), with x(a) the drift from a_i to a. x_i already carries the replicate offset. Returns
    (a_L, x(a_L)), or None when the image does not change side of the lightcone in the step."""
    o = np.asarray(origin, dtype=np.float64)

    def position(a):
        q, dd1, dd2 = partial_drift(a_i, a, a_ip1, omega_m, modified, n_lpt)
        x = x_i + q * p
        if cola:
            x = x + dd1 * psi1 + dd2 * psi2
        return x

    g = lambda a: np.sqrt(np.sum((position(a) - o) ** 2)) - comoving_distance(a, omega_m)
    if not (g(a_i) <= 0.0 < g(a_ip1)):
        return None
    a_l = optimize.brentq(g, a_i, a_ip1, xtol=1e-14, rtol=1e-14)
    return a_l, position(a_l)


def lightcone_run(pos, vel, psi1, psi2, a_list, omega_m, n_mesh, box, origin, a_start, rep_lo=(0, 0, 0),
                  rep_hi=(0, 0, 0), cola=True, modified=True, n_lpt=-2.5, deconv_power=1, force_fn=None):
    """The COLA run of oracle.cola.cola_run with the lightcone drift of Sec. 6.1. Returns (pos, vel, records), the
    records the concatenated drift_crossings of every lightcone drift."""
    if force_fn is None:
        force_fn = lambda x, a: pm_force(x, n_mesh, box, deconv_power)
    x = np.array(pos, dtype=np.float64)
    p = np.array(vel, dtype=np.float64)
    psi1 = np.asarray(psi1, dtype=np.float64)
    psi2 = np.asarray(psi2, dtype=np.float64)
    tab = cosmo.coefficient_table(a_list, omega_m, modified, n_lpt)
    col = {name: k for k, name in enumerate(cosmo.COEF_COLUMNS)}
    if cola:
        p = p - (tab[0, col["f1"]] * psi1 + tab[0, col["f2"]] * psi2)
    n_last = tab.shape[0] - 1
    records = []
    for i in range(n_last + 1):
        row = tab[i]
        g = force_fn(x, row[col["a"]])
        acc = kick_acceleration(g, psi1, psi2, omega_m, row[col["D1"]], row[col["D2"]], cola)
        p = p + row[col["K"]] * acc
        if i < n_last:
            a_i, a_ip1 = row[col["a"]], tab[i + 1, col["a"]]
            if a_i >= a_start:
                records.append(drift_crossings(x, p, psi1, psi2, a_i, a_ip1, omega_m, box, origin, rep_lo, rep_hi,
                                               cola, modified, n_lpt))
            x = x + row[col["Q"]] * p
            if cola:
                x = x + row[col["dDD1"]] * psi1 + row[col["dDD2"]] * psi2
            x = np.mod(x, box)
    if cola:
        p = p + tab[n_last, col["f1"]] * psi1 + tab[n_last, col["f2"]] * psi2
    if records:
        rec = {k: np.concatenate([r[k] for r in records], axis=-1) for k in records[0]}
    else:
        rec = {"index": np.zeros(0, np.int64), "replicate": np.zeros(0, np.int64), "a": np.zeros(0),
               "pos": np.zeros((3, 0)), "vel": np.zeros((3, 0))}
    return x, p, rec


def active_replicates(box, rep_lo, rep_hi, origin, r_l):
    """Flat indices of the replicates whose cube [o, o + L)^3 has a point within r_l of the origin (Sec. 6.2.3: any
    replicate whose closest point lies beyond the lightcone radius has left the lightcone for good)."""
    offs, ids = replicate_offsets(box, rep_lo, rep_hi)
    o = np.asarray(origin, dtype=np.float64)
    d = np.maximum(0.0, np.maximum(offs - o, o - (offs + box)))  # per-axis distance from the origin to the cube
    return ids[np.sqrt(np.sum(d * d, axis=1)) <= r_l]
