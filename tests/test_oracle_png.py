"""Pins for oracle/png.py: the preset kernels reproduce the published bispectrum templates (local, equilateral,
orthogonal) for any tilt and any potential amplitude; the real-space construction of the non-linear term equals its
closed form on two plane waves for every preset and a generic term; fNL = 0 gives back the Gaussian field exactly; the
growth suppression equals the quadrature growth factor's early-time limit."""
import numpy as np
import pytest

import synth
from oracle import cosmology as oc
from oracle import ic as oic
from oracle import png

C = synth.COSMOLOGY


@pytest.mark.parametrize("kind", ["local", "equilateral", "orthogonal"])
@pytest.mark.parametrize("n_s", [1.0, 0.96])
def test_preset_kernels_give_the_templates(kind, n_s):
    rng = np.random.default_rng(1)
    k1 = rng.uniform(0.01, 0.3, 200)
    k2 = rng.uniform(0.01, 0.3, 200)
    k3 = np.abs(k1 - k2) + rng.uniform(0.0, 1.0, 200) * (k1 + k2 - np.abs(k1 - k2))  # triangle inequality
    amp = 3.7e-9
    p = lambda k: amp * k ** (n_s - 4.0)
    got = png.kernel_bispectrum(png.PRESETS[kind], k1, k2, k3, p, n_s)
    ref = png.template_bispectrum(kind, p(k1), p(k2), p(k3))
    assert np.allclose(got, ref, rtol=1e-11, atol=0)
    # all three shapes share the equilateral normalisation B(k, k, k) = 6 P(k)^2
    k = np.array([0.1])
    assert png.template_bispectrum(kind, p(k), p(k), p(k))[0] == pytest.approx(6 * p(k)[0] ** 2, rel=1e-12)


TERMS = {**png.PRESETS, "generic": [(0.7, 0.5, 1.5, -1.0), (-0.2, 2.0, 0.0, 0.0)]}


@pytest.mark.parametrize("kind", sorted(TERMS))
def test_nonlinear_term_plane_wave_closed_form(kind):
    """phi = A cos(k1.x) + B cos(k2.x): D^s cos(k.x) = m_s(|k|) cos(k.x), the products split into cos(2 k1.x),
    cos(2 k2.x), cos((k1 + k2).x), cos((k1 - k2).x) and a constant (dropped), and D^g scales each by m_g of its
    wavevector."""
    n, box, n_s, A, B = 16, 100.0, 0.96, 0.8, -1.3
    k1 = 2 * np.pi / box * np.array([1.0, 2.0, 0.0])
    k2 = 2 * np.pi / box * np.array([0.0, 1.0, 3.0])
    x = np.arange(n) * (box / n)
    X = np.stack(np.meshgrid(x, x, x, indexing="ij"))
    ph = lambda k: np.tensordot(k, X, axes=1)
    phi = A * np.cos(ph(k1)) + B * np.cos(ph(k2))
    got = np.fft.irfftn(png.nonlinear_term(np.fft.rfftn(phi), n, box, n_s, TERMS[kind]), s=(n,) * 3, axes=(0, 1, 2))
    m = lambda k, s: png.operator_power(np.linalg.norm(k), s, n_s) if s else 1.0
    ref = np.zeros_like(phi)
    for c, a, b, g in TERMS[kind]:
        ref += c * (A * A * m(k1, a) * m(k1, b) / 2 * m(2 * k1, g) * np.cos(ph(2 * k1))
                    + B * B * m(k2, a) * m(k2, b) / 2 * m(2 * k2, g) * np.cos(ph(2 * k2))
                    + A * B * (m(k1, a) * m(k2, b) + m(k2, a) * m(k1, b)) / 2
                    * (m(k1 + k2, g) * np.cos(ph(k1 + k2)) + m(k1 - k2, g) * np.cos(ph(k1 - k2))))
    assert np.allclose(got, ref, atol=1e-12 * np.abs(ref).max())


def test_zero_fnl_is_the_gaussian_field():
    n, box = 24, 200.0
    cosmo = dict(omega_m=C["omega_m"], h=C["h"], n_s=C["n_s"], sigma8=C["sigma8"])
    g = oic.gaussian_field_hat(4, n, box, **cosmo)
    for kind in png.PRESETS:
        d = png.delta_hat_png(4, n, box, **cosmo, f_nl=0.0, terms=png.PRESETS[kind])
        assert np.allclose(d, g, rtol=1e-12, atol=1e-12 * np.abs(g).max())
    d = png.delta_hat_png(4, n, box, **cosmo, f_nl=100.0, terms=png.PRESETS["local"])
    assert 1e-6 < np.abs(d - g).max() / np.abs(g).max() < 1e-2


def test_growth_suppression_is_the_early_time_limit():
    om = C["omega_m"]
    a = 1e-4
    assert png.growth_suppression(om) == pytest.approx(a / oc.growth_D1(a, om), rel=1e-6)
    assert png.growth_suppression(1.0) == 1.0


def test_local_fnl_skews_the_potential():
    """Phi - phi = fNL (phi^2 - <phi^2>) in real space for the local preset (up to the Nyquist planes), so a positive
    fNL makes Phi positively skewed."""
    n, box = 32, 400.0
    cosmo = dict(omega_m=C["omega_m"], h=C["h"], n_s=C["n_s"], sigma8=C["sigma8"])
    phi_hat = png.primordial_potential_hat(7, n, box, **cosmo)
    phi = np.fft.irfftn(phi_hat, s=(n,) * 3, axes=(0, 1, 2))
    nl = np.fft.irfftn(png.nonlinear_term(phi_hat, n, box, cosmo["n_s"], png.PRESETS["local"]), s=(n,) * 3, axes=(0, 1, 2))
    sq = np.fft.rfftn(phi**2 - np.mean(phi**2))
    k, zero = png._k_half(n, box)
    assert np.allclose(nl, np.fft.irfftn(np.where(zero, 0.0, sq), s=(n,) * 3, axes=(0, 1, 2)), atol=1e-12 * np.abs(nl).max())
    Phi = phi + 3e4 * nl
    skew = lambda f: np.mean((f - f.mean()) ** 3) / np.std(f) ** 3
    assert skew(Phi) > skew(phi) + 0.1
