"""Binned power spectrum of a periodic box, in float64.

Oracle (test infrastructure only). In a periodic cubic box with uniform mean density, the FKP estimator named in
Sec. 7.1 (and Sec. 6) reduces to the binned mean of |delta_hat|^2; shot noise is not subtracted (Sec. 7.1).

Readings taken: P(n) = V |delta_hat(n)|^2 / (M^2 W(n)^2) with M = Nm^3, V = L^3 and one CIC window
W = prod_d sinc^2(pi n_d / Nm) removed in amplitude; bins [b dk, (b+1) dk) with dk = k_max / n_bins on |k|, the
n = 0 mode excluded; each r2c-half mode with 0 < n_z < Nm/2 also stands for its Hermitian partner and is counted
twice. Each bin reports the mean |k|, the mean P and the mode count; empty bins report NaN.
"""
import numpy as np

from .pm import deposit_fixed, density_contrast


def binned_power_from_delta(delta, box, k_max, n_bins, window_power=2):
    """Binned P(k) of a real mesh field delta (shape (Nm,)*3) divided by W^window_power in power."""
    n_mesh = delta.shape[0]
    dk = k_max / n_bins
    dh = np.fft.rfftn(delta)
    nf = np.fft.fftfreq(n_mesh, d=1.0 / n_mesh)
    nh = np.arange(n_mesh // 2 + 1, dtype=np.float64)
    kf = 2.0 * np.pi / box
    k = kf * np.sqrt(nf[:, None, None] ** 2 + nf[None, :, None] ** 2 + nh[None, None, :] ** 2)
    wf = np.sinc(nf / n_mesh) ** 2
    wh = np.sinc(nh / n_mesh) ** 2
    W = wf[:, None, None] * wf[None, :, None] * wh[None, None, :]
    M = float(n_mesh) ** 3
    P = box**3 * np.abs(dh) ** 2 / (M * M) / W**window_power
    mult = np.where((nh > 0) & (nh < n_mesh / 2), 2.0, 1.0)[None, None, :] * np.ones_like(P)
    b = np.floor(k / dk).astype(np.int64)
    use = (k > 0.0) & (b < n_bins)
    cnt = np.bincount(b[use], weights=mult[use], minlength=n_bins)
    sk = np.bincount(b[use], weights=(mult * k)[use], minlength=n_bins)
    sp = np.bincount(b[use], weights=(mult * P)[use], minlength=n_bins)
    with np.errstate(invalid="ignore", divide="ignore"):
        kmean = np.where(cnt > 0, sk / np.where(cnt > 0, cnt, 1.0), np.nan)
        pmean = np.where(cnt > 0, sp / np.where(cnt > 0, cnt, 1.0), np.nan)
    return kmean, pmean, cnt.astype(np.int64)


def power_spectrum(pos, n_mesh, box, k_max, n_bins):
    """Deposit the particles (fixed-point CIC), then bin P(k) with the CIC window removed once in amplitude."""
    pos = np.asarray(pos)
    C = deposit_fixed(pos, n_mesh, box)
    return binned_power_from_delta(density_contrast(C, pos.shape[1]), box, k_max, n_bins, window_power=2)
