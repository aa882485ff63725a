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
