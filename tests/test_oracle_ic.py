"""Pins for oracle/rng.py and oracle/ic.py: SplitMix64 reference outputs, white-noise statistics, the two-wave 2LPT
closed form, the Zel'dovich divergence, the sigma8 normalisation and the measured IC power spectrum."""
import os

import numpy as np
import pytest
from scipy import integrate

from oracle import ic, rng

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "splitmix64_seed0.txt")
COSMO = dict(omega_m=0.31, h=0.68, n_s=0.96, sigma8=0.8)


def test_splitmix64_reference_outputs():
    rows = [l.split() for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    for c, hexval in rows:
        assert int(rng.splitmix64(0, int(c))) == int(hexval, 16)


def test_white_noise_statistics():
    g = rng.white_noise(42, 64).ravel()
    n = g.size
    assert abs(g.mean()) < 5 / np.sqrt(n)
    assert abs(g.var() - 1.0) < 5 * np.sqrt(2.0 / n)
    assert abs(np.mean(g**4) / g.var() ** 2 - 3.0) < 0.05
    assert abs(np.corrcoef(g[:-1], g[1:])[0, 1]) < 5 / np.sqrt(n)
    assert not np.array_equal(rng.white_noise(43, 8), rng.white_noise(42, 8))


def test_two_wave_2lpt_closed_form():
    """phi1 = A cos(kx x) + B cos(ky y)  =>  phi2 = -A B kx^2 ky^2 cos(kx x) cos(ky y) / (kx^2 + ky^2)."""
    n, box, A, B = 16, 100.0, 3.0, -2.0
    kx, ky = 2 * np.pi * 2 / box, 2 * np.pi * 3 / box
    x = np.arange(n) * (box / n)
    X, Y, _ = np.meshgrid(x, x, x, indexing="ij")
    delta = -A * kx**2 * np.cos(kx * X) - B * ky**2 * np.cos(ky * Y)       # lap phi1
    psi1, psi2 = ic.lpt_displacements(np.fft.rfftn(delta), n, box)
    assert np.allclose(psi1[0], A * kx * np.sin(kx * X), atol=1e-12)
    assert np.allclose(psi1[1], B * ky * np.sin(ky * Y), atol=1e-12)
    assert np.allclose(psi1[2], 0.0, atol=1e-12)
    c = A * B * kx**2 * ky**2 / (kx**2 + ky**2)
    assert np.allclose(psi2[0], c * kx * np.sin(kx * X) * np.cos(ky * Y), atol=1e-12)
    assert np.allclose(psi2[1], c * ky * np.cos(kx * X) * np.sin(ky * Y), atol=1e-12)
    assert np.allclose(psi2[2], 0.0, atol=1e-12)


def test_zeldovich_divergence_is_minus_delta():
    n, box = 16, 64.0
    dh = ic.gaussian_field_hat(5, n, box, **COSMO)
    psi1, _ = ic.lpt_displacements(dh, n, box)
    nf = np.fft.fftfreq(n, d=1.0 / n) * 2 * np.pi / box
    nh = np.arange(n // 2 + 1) * 2 * np.pi / box
    ks = (nf[:, None, None], nf[None, :, None], nh[None, None, :])
    div_hat = sum(1j * ks[j] * np.fft.rfftn(psi1[j]) for j in range(3))
    assert np.allclose(div_hat, -dh, atol=1e-9 * np.abs(dh).max())


def test_sigma8_normalisation_independent_quadrature():
    """Integrate sigma8^2 again, in k (not ln k), with a fixed 4000-point Gauss-Legendre rule per decade."""
    A = ic.pk_amplitude(**COSMO)
    xg, wg = np.polynomial.legendre.leggauss(400)
    total = 0.0
    for lo, hi in zip(10.0 ** np.arange(-6, 3), 10.0 ** np.arange(-5, 4)):
        for a, b in zip(np.linspace(lo, hi, 11)[:-1], np.linspace(lo, hi, 11)[1:]):
            k = 0.5 * (b - a) * xg + 0.5 * (a + b)
            f = k**2 * A * ic.unnormalised_pk(k, COSMO["omega_m"], COSMO["h"], COSMO["n_s"]) * ic.tophat_window(8 * k) ** 2
            total += 0.5 * (b - a) * np.sum(wg * f)
    assert np.sqrt(total / (2 * np.pi**2)) == pytest.approx(0.8, rel=1e-10)


def test_tophat_and_transfer_limits():
    assert ic.tophat_window(1e-5) == pytest.approx(1.0, abs=1e-10)
    x = 2.0
    assert ic.tophat_window(x) == pytest.approx(3 * (np.sin(x) - x * np.cos(x)) / x**3, rel=1e-14)
    assert ic.bbks_transfer(1e-8, 0.31, 0.68) == pytest.approx(1.0, abs=1e-6)
    t = ic.bbks_transfer(np.logspace(-3, 1, 50), 0.31, 0.68)
    assert np.all(np.diff(t) < 0) and np.all(t > 0)


def test_ic_field_has_input_power():
    """The discrete field's |delta_hat|^2 V / N^6, averaged in shells, equals P(k) within cosmic variance."""
    n, box = 48, 300.0
    dh = ic.gaussian_field_hat(11, n, box, **COSMO)
    nf = np.fft.fftfreq(n, d=1.0 / n)
    nh = np.arange(n // 2 + 1)
    kmag = 2 * np.pi / box * np.sqrt(nf[:, None, None] ** 2 + nf[None, :, None] ** 2 + nh[None, None, :] ** 2)
    P = np.abs(dh) ** 2 * box**3 / n**6
    ratio = P / ic.linear_pk(np.where(kmag == 0, 1.0, kmag), **COSMO)
    edges = np.linspace(0.05, 0.45, 5)
    for lo, hi in zip(edges[:-1], edges[1:]):
        sel = (kmag >= lo) & (kmag < hi) & (P > 0)
        m = sel.sum()
        assert abs(ratio[sel].mean() - 1.0) < 5 * np.sqrt(1.0 / m)


def test_initial_conditions_layout():
    out = ic.initial_conditions(1, 8, 64.0, 0.1, **COSMO)
    assert out["pos"].shape == (3, 512) and out["id"][5] == 5
    q = ic.lattice_positions(8, 64.0)
    assert np.array_equal(q[:, 1], [4.0, 4.0, 12.0]) and np.array_equal(q[:, 8], [4.0, 12.0, 4.0])
    assert np.all((out["pos"] >= 0) & (out["pos"] <= 64.0))


def _two_wave_fields(n, box, A, B):
    """Psi1, Psi2 of the two-wave potential phi1 = A cos(kx x) + B cos(ky y), from lpt_displacements (pinned above
    by its closed form), on the cell-centred lattice the particles start from."""
    kx, ky = 2 * np.pi * 2 / box, 2 * np.pi * 3 / box
    x = (np.arange(n) + 0.5) * (box / n)
    X, Y, _ = np.meshgrid(x, x, x, indexing="ij")
    delta = -A * kx**2 * np.cos(kx * X) - B * ky**2 * np.cos(ky * Y)
    return ic.lpt_displacements(np.fft.rfftn(delta), n, box)


@pytest.mark.parametrize("a0", [0.1, 0.37])
def test_ic_assembly_einstein_de_sitter_closed_form(a0):
    """Omega_m = 1: D1 = a, D2 = -3/7 a^2, E = a^-3/2, so x = q + a Psi1 - (3/7) a^2 Psi2 and
    p = a^3 E (D1' Psi1 + D2' Psi2) = a^(3/2) Psi1 - (6/7) a^(5/2) Psi2, element by element."""
    n, box = 16, 100.0
    psi1, psi2 = _two_wave_fields(n, box, 3.0, -2.0)
    out = ic.particles_from_displacements(psi1, psi2, n, box, a0, 1.0)
    p1, p2 = psi1.reshape(3, -1), psi2.reshape(3, -1)
    assert np.abs(p2).max() > 1e-3  # the second-order field is not trivially zero
    q = ic.lattice_positions(n, box)
    x_ref = np.mod(q + a0 * p1 - 3.0 / 7.0 * a0**2 * p2, box)
    d = out["pos"] - x_ref
    d -= box * np.round(d / box)
    assert np.abs(d).max() < 1e-10
    v_ref = a0**1.5 * p1 - 6.0 / 7.0 * a0**2.5 * p2
    assert np.allclose(out["vel"], v_ref, rtol=0, atol=1e-10 * np.abs(v_ref).max())
    assert np.array_equal(out["psi1"], p1) and np.array_equal(out["psi2"], p2)


def test_ic_momentum_is_the_cola_frame_momentum():
    """With the force that the 2LPT trajectory itself feels, g = -(D1 Psi1 + (D2 - D1^2) Psi2), the COLA residual
    acceleration vanishes. The IC momentum minus the frame momentum the integrator removes must then be exactly zero,
    so the run follows x(a) = q + D1(a) Psi1 + D2(a) Psi2 and ends with the frame momentum of its last time. A sign
    slip on the D2 term, or a frame momentum at the wrong time, moves x by Q p_res and fails this."""
    from oracle import cola as ocola
    from oracle import cosmology as oc
    n, box, om = 8, 64.0, 1.0
    psi1, psi2 = _two_wave_fields(n, box, 4.0, 2.5)
    a_list = [0.1, 0.3, 0.55, 1.0]
    out = ic.particles_from_displacements(psi1, psi2, n, box, a_list[0], om)
    p1, p2 = out["psi1"], out["psi2"]

    def lpt_force(x, a):
        d1, d2 = oc.growth_D1(a, om), oc.growth_D2(a, om)
        return -(d1 * p1 + (d2 - d1 * d1) * p2)

    x, p = ocola.cola_run(out["pos"], out["vel"], p1, p2, a_list, om, n, box, force_fn=lpt_force)
    aN = a_list[-1]
    q = ic.lattice_positions(n, box)
    d = x - np.mod(q + aN * p1 - 3.0 / 7.0 * aN**2 * p2, box)
    d -= box * np.round(d / box)
    assert np.abs(d).max() < 1e-9
    assert np.allclose(p, aN**1.5 * p1 - 6.0 / 7.0 * aN**2.5 * p2, rtol=0, atol=1e-9)
