"""Initial conditions with primordial non-Gaussianity, in float64.

Oracle (test infrastructure only). Sec. 5 of Howlett, Manera & Percival (2015): the initial conditions can carry local,
equilateral, orthogonal or generic primordial non-Gaussianity of amplitude fNL, the generic case given by a kernel in
the formalism of Scoccimarro et al. (2012). The paper states no formula; the readings below define one.

  * Gaussian primordial potential phi with power P_phi(k) = A k^(ns - 4) / alpha0^2, drawn from the same white noise
    as the Gaussian initial conditions: phi_hat = noise_hat sqrt(P_phi N^3 / V), with the k = 0 mode and every Nyquist
    plane zeroed.
  * Phi = phi + fNL (NL[phi] - <NL[phi]>) with NL[phi] = sum_j c_j D^g_j[(D^a_j phi) (D^b_j phi)], where D^s multiplies
    Fourier mode k by (P_phi(k) / A_phi)^(-s/3) = k^(s (4 - ns) / 3) (k in h/Mpc), i.e. by |k|^s for a scale-invariant
    spectrum. For a kernel whose exponents sum to zero (a + b + g = 0 in every term) the leading-order bispectrum of
    Phi is 2 fNL sum over the three pairs of K(k1, k2) P1 P2 with K the symmetrised kernel, and the fractional powers
    of P of the standard templates come out exactly, at any tilt.
  * Presets: local NL = phi^2; equilateral (Creminelli et al. 2006) NL = -3 phi^2 + 6 D^-1[(D phi) phi]
    - 2 D^-2[(D phi)^2]; orthogonal (Senatore et al. 2010) NL = -9 phi^2 + 18 D^-1[(D phi) phi] - 8 D^-2[(D phi)^2].
    These coefficients follow from matching the kernel's bispectrum to each template (pinned in the tests).
  * Phi is the primordial Bardeen potential with the sign of the curvature perturbation (positive fNL: positively
    skewed density), linked to the linear density at z = 0 by delta(k) = alpha(k) Phi(k),
    alpha(k) = (2/3) (c/H0)^2 k^2 T(k) g0 / Om, with g0 = D1(1) / lim_{a->0} (D1(a)/a) the growth suppression of the
    normalisation D1(1) = 1 (g0 = 2F1(1/3, 1; 11/6; -OL/Om) for flat LCDM); alpha0 = (2/3) (c/H0)^2 g0 / Om so that
    alpha(k)^2 P_phi(k) = A k^ns T^2, the Gaussian spectrum: fNL = 0 gives back the Gaussian initial conditions.
  * The k = 0 mode and the Nyquist planes of Phi_hat are zeroed (the mean subtraction); the 2LPT displacements then
    follow as in oracle.ic.
"""
import numpy as np
from scipy.special import hyp2f1

from . import ic
from .rng import white_noise

C_OVER_H0 = 2997.92458  # Mpc/h

# (c, a, b, g) per term of NL[phi] = sum c D^g[(D^a phi)(D^b phi)]
PRESETS = {
    "local": [(1.0, 0.0, 0.0, 0.0)],
    "equilateral": [(-3.0, 0.0, 0.0, 0.0), (6.0, 1.0, 0.0, -1.0), (-2.0, 1.0, 1.0, -2.0)],
    "orthogonal": [(-9.0, 0.0, 0.0, 0.0), (18.0, 1.0, 0.0, -1.0), (-8.0, 1.0, 1.0, -2.0)],
}


def growth_suppression(omega_m):
    """g0 = D1(1) / lim_{a->0} (D1(a) / a) for D1(1) = 1 (flat LCDM closed form)."""
    return float(hyp2f1(1.0 / 3.0, 1.0, 11.0 / 6.0, -(1.0 - omega_m) / omega_m))


def potential_to_density(k, omega_m, h):
    """alpha(k) with delta_L(k, z = 0) = alpha(k) Phi(k)."""
    g0 = growth_suppression(omega_m)
    return (2.0 / 3.0) * C_OVER_H0**2 * np.asarray(k) ** 2 * ic.bbks_transfer(k, omega_m, h) * g0 / omega_m


def _k_half(n, box):
    nf = np.fft.fftfreq(n, d=1.0 / n)
    nh = np.arange(n // 2 + 1, dtype=np.float64)
    kf = 2.0 * np.pi / box
    k = kf * np.sqrt(nf[:, None, None] ** 2 + nf[None, :, None] ** 2 + nh[None, None, :] ** 2)
    nyq = (np.abs(nf)[:, None, None] == n // 2) | (np.abs(nf)[None, :, None] == n // 2) | (nh[None, None, :] == n // 2)
    return k, nyq | (k == 0.0)


def operator_power(k, s, n_s):
    """The Fourier multiplier of D^s: k^(s (4 - ns) / 3), and 0 at k = 0."""
    k = np.asarray(k, dtype=np.float64)
    return np.where(k > 0.0, np.where(k > 0.0, k, 1.0) ** (s * (4.0 - n_s) / 3.0), 0.0)


def primordial_potential_hat(seed, n_side, box, omega_m, h, n_s, sigma8):
    """phi_hat (r2c half, unnormalised DFT) with the power A k^(ns-4) / alpha0^2 of the Gaussian potential."""
    k, zero = _k_half(n_side, box)
    amp = ic.pk_amplitude(omega_m, h, n_s, sigma8)
    alpha0 = (2.0 / 3.0) * C_OVER_H0**2 * growth_suppression(omega_m) / omega_m
    p_phi = amp * np.where(zero, 1.0, k) ** (n_s - 4.0) / alpha0**2
    noise_hat = np.fft.rfftn(white_noise(seed, n_side))
    return np.where(zero, 0.0, noise_hat * np.sqrt(p_phi * n_side**3 / box**3))


def nonlinear_term(phi_hat, n_side, box, n_s, terms):
    """NL[phi]_hat (half spectrum) = sum_j c_j D^g_j[(D^a_j phi)(D^b_j phi)], k = 0 and Nyquist zeroed."""
    k, zero = _k_half(n_side, box)
    shape = (n_side,) * 3
    out = np.zeros_like(phi_hat)
    for c, a, b, g in terms:
        fa = np.fft.irfftn(phi_hat * operator_power(k, a, n_s) if a else phi_hat, s=shape, axes=(0, 1, 2))
        fb = np.fft.irfftn(phi_hat * operator_power(k, b, n_s) if b else phi_hat, s=shape, axes=(0, 1, 2))
        prod_hat = np.fft.rfftn(fa * fb)
        out = out + c * (prod_hat * operator_power(k, g, n_s) if g else prod_hat)
    return np.where(zero, 0.0, out)


def delta_hat_png(seed, n_side, box, omega_m, h, n_s, sigma8, f_nl, terms):
    """delta_L_hat = alpha(k) (phi_hat + fNL NL_hat), Nyquist planes and k = 0 zeroed."""
    phi_hat = primordial_potential_hat(seed, n_side, box, omega_m, h, n_s, sigma8)
    Phi_hat = phi_hat + f_nl * nonlinear_term(phi_hat, n_side, box, n_s, terms)
    k, zero = _k_half(n_side, box)
    return np.where(zero, 0.0, potential_to_density(np.where(zero, 1.0, k), omega_m, h) * Phi_hat)


def initial_conditions_png(seed, n_side, box, a_init, omega_m, h, n_s, sigma8, f_nl, terms):
    """oracle.ic.initial_conditions with the non-Gaussian linear field of delta_hat_png."""
    delta_hat = delta_hat_png(seed, n_side, box, omega_m, h, n_s, sigma8, f_nl, terms)
    psi1, psi2 = ic.lpt_displacements(delta_hat, n_side, box)
    return ic.particles_from_displacements(psi1, psi2, n_side, box, a_init, omega_m)


def template_bispectrum(kind, p1, p2, p3):
    """The published shapes per unit fNL, in terms of the three potential powers (local: 2 sum of pair products)."""
    pairs = p1 * p2 + p2 * p3 + p3 * p1
    if kind == "local":
        return 2.0 * pairs
    cube = (p1 * p2 * p3) ** (2.0 / 3.0)
    ps = (p1, p2, p3)
    six = sum(ps[i] ** (1.0 / 3.0) * ps[j] ** (2.0 / 3.0) * ps[l] for i in range(3) for j in range(3) for l in range(3)
              if len({i, j, l}) == 3)
    if kind == "equilateral":
        return 6.0 * (-pairs - 2.0 * cube + six)
    if kind == "orthogonal":
        return 6.0 * (-3.0 * pairs - 8.0 * cube + 3.0 * six)
    raise ValueError(kind)


def kernel_bispectrum(terms, k1, k2, k3, p_of_k, n_s):
    """2 sum over the three pairs of K_sym(ki, kj) Pi Pj, with K_sym the symmetrised kernel of the terms (per unit
    fNL, leading order)."""
    ks = (k1, k2, k3)
    P = [p_of_k(k) for k in ks]
    m = lambda k, s: operator_power(k, s, n_s)
    total = 0.0
    for (i, j, l) in ((0, 1, 2), (1, 2, 0), (2, 0, 1)):
        K = sum(c * m(ks[l], g) * 0.5 * (m(ks[i], a) * m(ks[j], b) + m(ks[i], b) * m(ks[j], a)) for c, a, b, g in terms)
        total = total + 2.0 * K * P[i] * P[j]
    return total
