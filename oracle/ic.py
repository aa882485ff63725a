"""Initial conditions: linear power spectrum, Gaussian field and 2LPT displacements on the particle lattice.

Oracle (test infrastructure only). Follows Sec. 2.1 (Eqs. 5-10: Zel'dovich and 2LPT displacements from the two
Lagrangian potentials) and Sec. 5 (displacements generated at the lattice points; particles created just before
timestepping) of Howlett, Manera & Percival (2015).

Readings taken (the paper uses CAMB and 2LPTic, neither of which is reproducible here):
  * P(k) = A k^ns T(k)^2 with the BBKS transfer function of Bardeen et al. (1986), q = k / Gamma, Gamma = Om h
    (k in h/Mpc), no baryon correction. A is fixed by sigma8 with the real-space top-hat of radius 8 Mpc/h.
    The BBKS constants are retyped from the published fit: parity unpinned (no printed value to check against).
  * delta_hat(n) = white_noise_hat(n) * sqrt(P(|k|) N^3 / V): the unnormalised DFT convention, so that the discrete
    field has the continuum power spectrum P. The n = 0 mode and every mode with a Nyquist index (|n_d| = N/2 on any
    axis) are set to zero, in delta_hat and in the 2LPT source spectrum.
  * Psi1 = -grad phi1 with lap phi1 = delta_L (Eqs. 8-9); Psi2 = grad phi2 with lap phi2 = the sum over i > j of
    (phi1_ii phi1_jj - phi1_ij^2) (Eq. 10). Positions x = q + D1 Psi1 + D2 Psi2 with D2 < 0 (Eq. 7), at the
    cell-centred lattice q = (i + 1/2, j + 1/2, l + 1/2) L / N ("a grid pattern", Sec. 5; the half-spacing offset
    puts the unperturbed particles at mesh-cell centres whenever Nm / N is odd, which keeps the CIC deposit linear in
    small displacements). Psi1 and Psi2 are the z = 0 (D1 = 1) displacements.
  * Momentum p = a^3 E (D1' Psi1 + D2' Psi2) (the LPT frame momentum).
"""
import functools

import numpy as np
from scipy import integrate

from . import cosmology as cosmo
from .rng import white_noise


def bbks_transfer(k, omega_m, h):
    """BBKS transfer function T(k), k in h/Mpc, shape parameter Gamma = Om h."""
    q = np.asarray(k, dtype=np.float64) / (omega_m * h)
    q = np.where(q == 0.0, 1e-300, q)
    x = 2.34 * q
    poly = 1.0 + 3.89 * q + (16.1 * q) ** 2 + (5.46 * q) ** 3 + (6.71 * q) ** 4
    return np.log1p(x) / x * poly**-0.25


def tophat_window(x):
    """Fourier transform of the real-space spherical top-hat: 3 (sin x - x cos x) / x^3."""
    x = np.asarray(x, dtype=np.float64)
    small = np.abs(x) < 1e-3
    xs = np.where(small, 1.0, x)
    w = 3.0 * (np.sin(xs) - xs * np.cos(xs)) / xs**3
    return np.where(small, 1.0 - x**2 / 10.0, w)


def unnormalised_pk(k, omega_m, h, n_s):
    k = np.asarray(k, dtype=np.float64)
    return k**n_s * bbks_transfer(k, omega_m, h) ** 2


def sigma_R(pk_fn, R):
    """sigma(R)^2 = (1 / 2 pi^2) int k^2 P(k) W(kR)^2 dk, integrated over ln k with adaptive quadrature."""
    f = lambda lnk: np.exp(lnk) ** 3 * pk_fn(np.exp(lnk)) * tophat_window(np.exp(lnk) * R) ** 2
    edges = np.linspace(np.log(1e-7), np.log(1e3), 81)
    rough = sum(integrate.quad(f, lo, hi, limit=200)[0] for lo, hi in zip(edges[:-1], edges[1:]))
    val = 0.0
    for lo, hi in zip(edges[:-1], edges[1:]):
        v, _ = integrate.quad(f, lo, hi, epsabs=1e-15 * rough, epsrel=1e-13, limit=400)
        val += v
    return np.sqrt(val / (2.0 * np.pi**2))


@functools.lru_cache(maxsize=32)
def pk_amplitude(omega_m, h, n_s, sigma8):
    """Amplitude A with sigma(8 Mpc/h) = sigma8 for P = A k^ns T^2."""
    s = sigma_R(lambda k: unnormalised_pk(k, omega_m, h, n_s), 8.0)
    return (sigma8 / s) ** 2


def linear_pk(k, omega_m, h, n_s, sigma8):
    return pk_amplitude(omega_m, h, n_s, sigma8) * unnormalised_pk(k, omega_m, h, n_s)


def wavenumbers(n, box):
    """Signed integer frequencies and k = 2 pi n / L for a full axis and for the r2c half axis."""
    nf = np.fft.fftfreq(n, d=1.0 / n)            # 0, 1, ..., n/2-1, -n/2, ..., -1
    nh = np.arange(n // 2 + 1, dtype=np.float64)  # 0 .. n/2
    return nf, nh, 2.0 * np.pi / box


def _k_grids(n, box):
    nf, nh, kf = wavenumbers(n, box)
    kx = (kf * nf)[:, None, None]
    ky = (kf * nf)[None, :, None]
    kz = (kf * nh)[None, None, :]
    nyq = (np.abs(nf)[:, None, None] == n // 2) | (np.abs(nf)[None, :, None] == n // 2) | (nh[None, None, :] == n // 2)
    k2 = kx**2 + ky**2 + kz**2
    zero = nyq | (k2 == 0.0)
    return kx, ky, kz, k2, zero


def gaussian_field_hat(seed, n_side, box, omega_m, h, n_s, sigma8):
    """delta_L in Fourier space (r2c half, unnormalised DFT convention), shape (N, N, N/2+1)."""
    noise_hat = np.fft.rfftn(white_noise(seed, n_side))
    kx, ky, kz, k2, zero = _k_grids(n_side, box)
    kmag = np.sqrt(k2)
    amp = np.sqrt(linear_pk(np.where(zero, 1.0, kmag), omega_m, h, n_s, sigma8) * n_side**3 / box**3)
    return np.where(zero, 0.0, noise_hat * amp)


def lpt_displacements(delta_hat, n_side, box):
    """Psi1 and Psi2 (each shape (3, N, N, N)) from the linear field delta_L, via Eqs. 8-10."""
    kx, ky, kz, k2, zero = _k_grids(n_side, box)
    ks = (kx, ky, kz)
    inv_k2 = np.where(zero, 0.0, 1.0 / np.where(k2 == 0.0, 1.0, k2))
    d = np.where(zero, 0.0, delta_hat)
    shape = (n_side,) * 3
    # phi1_hat = -delta_hat / k^2 ; Psi1 = -grad phi1  ->  Psi1_hat_j = -i k_j phi1_hat = i k_j delta_hat / k^2
    phi1_hat = -d * inv_k2
    psi1 = np.stack([np.fft.irfftn(-1j * ks[j] * phi1_hat, s=shape, axes=(0, 1, 2)) for j in range(3)])
    # second derivatives phi1_ij = IFFT(-k_i k_j phi1_hat)
    phi = {}
    for i in range(3):
        for j in range(i, 3):
            phi[i, j] = np.fft.irfftn(-ks[i] * ks[j] * phi1_hat, s=shape, axes=(0, 1, 2))
    src = (phi[0, 0] * phi[1, 1] + phi[0, 0] * phi[2, 2] + phi[1, 1] * phi[2, 2]
           - phi[0, 1] ** 2 - phi[0, 2] ** 2 - phi[1, 2] ** 2)
    src_hat = np.where(zero, 0.0, np.fft.rfftn(src))
    phi2_hat = -src_hat * inv_k2                  # lap phi2 = src
    psi2 = np.stack([np.fft.irfftn(1j * ks[j] * phi2_hat, s=shape, axes=(0, 1, 2)) for j in range(3)])  # Psi2 = +grad phi2
    return psi1, psi2


def lattice_positions(n_side, box):
    """q = (i + 1/2, j + 1/2, l + 1/2) L / N for lattice index (i N + j) N + l, shape (3, N^3)."""
    g = (np.arange(n_side, dtype=np.float64) + 0.5) * (box / n_side)
    qx, qy, qz = np.meshgrid(g, g, g, indexing="ij")
    return np.stack([qx.ravel(), qy.ravel(), qz.ravel()])


def particles_from_displacements(psi1, psi2, n_side, box, a_init, omega_m):
    """The particles at a_init from the z = 0 displacement fields (each (3, N, N, N) or (3, N^3)), Sec. 2.1 Eq. 5 and
    Sec. 2.2: x = q + D1(a) Psi1 + D2(a) Psi2 wrapped into [0, L), and the momentum of the 2LPT trajectory,
    p = a^2 dx/dt / H0 = a^3 E(a) (D1'(a) Psi1 + D2'(a) Psi2). Returns the dict of initial_conditions."""
    npart = n_side**3
    psi1 = np.asarray(psi1, dtype=np.float64).reshape(3, npart)
    psi2 = np.asarray(psi2, dtype=np.float64).reshape(3, npart)
    d1 = cosmo.growth_D1(a_init, omega_m)
    d2 = cosmo.growth_D2(a_init, omega_m)
    f1, f2 = cosmo.frame_momentum_factors(a_init, omega_m)
    pos = np.mod(lattice_positions(n_side, box) + d1 * psi1 + d2 * psi2, box)
    vel = f1 * psi1 + f2 * psi2
    return {"pos": pos, "vel": vel, "psi1": psi1, "psi2": psi2, "id": np.arange(npart, dtype=np.int64)}


def initial_conditions(seed, n_side, box, a_init, omega_m, h, n_s, sigma8):
    """2LPT particles at a_init. Returns dict of float64 arrays pos, vel, psi1, psi2 (each (3, N^3)) and id (N^3,)."""
    delta_hat = gaussian_field_hat(seed, n_side, box, omega_m, h, n_s, sigma8)
    psi1, psi2 = lpt_displacements(delta_hat, n_side, box)
    return particles_from_displacements(psi1, psi2, n_side, box, a_init, omega_m)
