"""Pins for oracle/spectrum.py: a planted single mode, mode counting, and the shot-noise level of uniform particles."""
import numpy as np
import pytest

import synth
from oracle import spectrum


def test_planted_mode_value_and_count():
    """delta = A cos(2 pi m x / L) on the mesh: |delta_hat|^2 = (A M / 2)^2 at +-m, so P = V A^2 / 4 / W(m)^2 there."""
    n, box, A, m = 32, 200.0, 0.3, 3
    x = np.arange(n)
    delta = A * np.cos(2 * np.pi * m * x / n)[None, None, :] * np.ones((n, n, 1))
    kf = 2 * np.pi / box
    dk = 3 * kf / 10.5                               # bin 10 = [2.857, 3.143) kf holds only |n|^2 = 9
    k, P, cnt = spectrum.binned_power_from_delta(delta, box, 11 * dk, 11, window_power=0)
    b = 10
    # |n|^2 = 9: the 6 axis modes (3,0,0) and the 24 modes (2,2,1) up to signs and order
    assert cnt[b] == 30
    assert k[b] == pytest.approx(3 * kf, rel=1e-14)
    # only n = (0, 0, +-3) carries power: the bin mean is 2/30 of V A^2 / 4
    assert P[b] == pytest.approx(box**3 * A**2 / 4 * 2 / 30, rel=1e-12)
    Pw = spectrum.binned_power_from_delta(delta, box, 11 * dk, 11, window_power=2)[1]
    assert Pw[b] == pytest.approx(P[b] / np.sinc(m / n) ** 4, rel=1e-12)
    # empty bins are NaN; total mode count equals the number of modes with 0 < |k| < k_max
    assert np.isnan(P[0]) and cnt[0] == 0


def test_total_mode_count_matches_full_grid():
    n, box = 16, 100.0
    k_max = 2 * np.pi / box * 6.5
    _, _, cnt = spectrum.binned_power_from_delta(np.zeros((n, n, n)), box, k_max, 13)
    f = np.fft.fftfreq(n, d=1.0 / n)
    kk = np.sqrt(f[:, None, None] ** 2 + f[None, :, None] ** 2 + f[None, None, :] ** 2) * 2 * np.pi / box
    assert cnt.sum() == np.count_nonzero((kk > 0) & (kk < k_max))


def test_uniform_particles_give_shot_noise():
    """Uniform random particles: P ~ 1/nbar = V / n at k well below the mesh Nyquist frequency."""
    n_part, box, n_mesh = 200_000, 100.0, 32
    pos = synth.uniform_positions(9, n_part, box).astype(np.float64)
    k, P, cnt = spectrum.power_spectrum(pos, n_mesh, box, 0.6, 6)
    sel = (k > 0.1) & (k < 0.6)
    assert np.all(np.abs(P[sel] / (box**3 / n_part) - 1.0) < 0.2)
