"""Particle-mesh force: fixed-point CIC deposit, FFT Poisson solve with CIC deconvolution, gradient, CIC gather.

Oracle (test infrastructure only). Follows the four steps of Sec. 2.4 (Eqs. 20-21) and the "round down to the cell"
cloud-in-cell of Sec. 4.2 of Howlett, Manera & Percival (2015).

Readings taken:
  * Mesh nodes sit at i * L / Nm. A particle whose coordinate lies in [i, i+1) cells gives weights (1 - f, f) to nodes
    i and i + 1 (periodic), f the fractional part, on each axis (Sec. 4.2, "rounding down").
  * The deposit is exact integer arithmetic with F = 16 fractional bits per axis: u = floor(x * (Nm 2^F / L)) taken
    in float64 (Nm 2^F / L itself a single float64 division), reduced mod Nm 2^F; i = u >> F, f = u & (2^F - 1);
    corner weights are products of (2^F - f) or f over the three axes, so each particle adds exactly 2^(3F).
  * Density in mean-density units: rho = C m 2^(-3F) with m = Nm^3 / n_particles; the FFT acts on delta = rho - 1
    (Sec. 2.2, Eq. 13: "rho(x) - 1").
  * Poisson: lap(psi) = delta, so psi_hat = -delta_hat / k^2 with the continuum k (Eq. 20, read with the sign and
    the 3/2 Om / a factor moved into the kick). Gradient: g_hat_j = i k_j psi_hat (Eq. 21 "k phi", read as the
    spectral derivative). CIC deconvolution: divide by W(n)^p, W = prod_d sinc^2(pi n_d / Nm). The paper deconvolves
    "the" CIC window once (Sec. 2.4, step 3), so p = 1 by default; p = 0 and p = 2 (deposit and gather windows) are
    also accepted. p = 2 amplifies particle-lattice discreteness on meshes finer than the particle spacing. The n = 0 mode and, for component j, the Nyquist plane
    n_j = Nm/2 are set to zero.
  * Gather: the transpose of the deposit, with weights f 2^-F and 1 - f 2^-F from the same fixed-point fractions.
"""
import numpy as np

FRAC_BITS = 16


def fixed_point_coords(pos, n_mesh, box, frac_bits=FRAC_BITS):
    """Integer cell index i and fraction f (both int64, shape (3, n)) of each particle coordinate."""
    scale = (float(n_mesh) * float(2**frac_bits)) / float(box)
    period = np.int64(n_mesh) << np.int64(frac_bits)
    u = np.floor(np.asarray(pos, dtype=np.float64) * scale).astype(np.int64)
    u = np.mod(u, period)  # numpy mod of int64 is non-negative for a positive period
    return u >> np.int64(frac_bits), u & np.int64((1 << frac_bits) - 1)


def deposit_fixed(pos, n_mesh, box, frac_bits=FRAC_BITS):
    """Fixed-point CIC density counts C (int64, shape (Nm, Nm, Nm)); sum(C) == n * 2^(3F) exactly."""
    idx, frac = fixed_point_coords(pos, n_mesh, box, frac_bits)
    one = np.int64(1 << frac_bits)
    C = np.zeros(n_mesh**3, dtype=np.int64)
    for cx in (0, 1):
        wx = frac[0] if cx else one - frac[0]
        ix = (idx[0] + cx) % n_mesh
        for cy in (0, 1):
            wy = frac[1] if cy else one - frac[1]
            iy = (idx[1] + cy) % n_mesh
            for cz in (0, 1):
                wz = frac[2] if cz else one - frac[2]
                iz = (idx[2] + cz) % n_mesh
                np.add.at(C, (ix * n_mesh + iy) * n_mesh + iz, wx * wy * wz)
    return C.reshape(n_mesh, n_mesh, n_mesh)


def fixed_point_overflow(pos, n_mesh, box, frac_bits=FRAC_BITS):
    """True when some cell's exact fixed-point count reaches 2^63, the headroom of a signed 64-bit count (the rule
    behind LPC_ERR_FIXED_OVERFLOW). Each corner weight w <= 2^(3F) is split into w >> 24 and w & (2^24 - 1); both
    per-cell sums fit int64 for any realistic particle count, and C = hi 2^24 + lo >= 2^63 exactly when
    hi + (lo >> 24) >= 2^39 (2^63 is a multiple of 2^24)."""
    idx, frac = fixed_point_coords(pos, n_mesh, box, frac_bits)
    one = np.int64(1 << frac_bits)
    hi = np.zeros(n_mesh**3, dtype=np.int64)
    lo = np.zeros(n_mesh**3, dtype=np.int64)
    for cx in (0, 1):
        wx = frac[0] if cx else one - frac[0]
        ix = (idx[0] + cx) % n_mesh
        for cy in (0, 1):
            wy = frac[1] if cy else one - frac[1]
            iy = (idx[1] + cy) % n_mesh
            for cz in (0, 1):
                wz = frac[2] if cz else one - frac[2]
                iz = (idx[2] + cz) % n_mesh
                w = wx * wy * wz
                cell = (ix * n_mesh + iy) * n_mesh + iz
                np.add.at(hi, cell, w >> np.int64(24))
                np.add.at(lo, cell, w & np.int64((1 << 24) - 1))
    return bool(np.any(hi + (lo >> np.int64(24)) >= np.int64(1 << 39)))


def density_contrast(C, n_particles, frac_bits=FRAC_BITS):
    """delta = C m 2^(-3F) - 1 with m = Nm^3 / n_particles (float64)."""
    m = C.size / float(n_particles)
    return C.astype(np.float64) * (m * 2.0 ** (-3 * frac_bits)) - 1.0


def cic_window(n_mesh):
    """Per-axis CIC window sinc^2(pi n / Nm) for the signed full axis and the r2c half axis."""
    nf = np.fft.fftfreq(n_mesh, d=1.0 / n_mesh)
    nh = np.arange(n_mesh // 2 + 1, dtype=np.float64)
    return np.sinc(nf / n_mesh) ** 2, np.sinc(nh / n_mesh) ** 2, nf, nh  # np.sinc(x) = sin(pi x)/(pi x)


def gradient_spectra(delta_hat, n_mesh, box, deconv_power=1):
    """g_hat_j = i k_j (-1/k^2) delta_hat / W^p for j = x, y, z (r2c half spectra)."""
    wf, wh, nf, nh = cic_window(n_mesh)
    kf = 2.0 * np.pi / box
    kx = (kf * nf)[:, None, None]
    ky = (kf * nf)[None, :, None]
    kz = (kf * nh)[None, None, :]
    k2 = kx**2 + ky**2 + kz**2
    W = wf[:, None, None] * wf[None, :, None] * wh[None, None, :]
    base = np.where(k2 == 0.0, 0.0, -1.0 / np.where(k2 == 0.0, 1.0, k2)) / W**deconv_power * delta_hat
    half = n_mesh // 2
    nyq = (np.abs(nf)[:, None, None] == half, np.abs(nf)[None, :, None] == half, nh[None, None, :] == half)
    out = []
    for j, k in enumerate((kx, ky, kz)):
        out.append(np.where(nyq[j], 0.0, 1j * k * base))
    return out


def force_mesh_from_delta(delta, box, deconv_power=1):
    """grad(psi) on the mesh, shape (3, Nm, Nm, Nm), for a real density-contrast mesh delta."""
    n_mesh = delta.shape[0]
    delta_hat = np.fft.rfftn(delta)
    spectra = gradient_spectra(delta_hat, n_mesh, box, deconv_power)
    return np.stack([np.fft.irfftn(s, s=delta.shape, axes=(0, 1, 2)) for s in spectra])


def force_mesh(C, n_particles, n_mesh, box, deconv_power=1):
    """grad(psi) on the mesh, shape (3, Nm, Nm, Nm), from fixed-point counts C."""
    return force_mesh_from_delta(density_contrast(C, n_particles), box, deconv_power)


def gather(mesh3, pos, n_mesh, box, frac_bits=FRAC_BITS):
    """CIC interpolation of a (3, Nm, Nm, Nm) field to particle positions, shape (3, n)."""
    idx, frac = fixed_point_coords(pos, n_mesh, box, frac_bits)
    f = frac.astype(np.float64) * 2.0**-frac_bits
    flat = mesh3.reshape(3, -1)
    out = np.zeros((3, idx.shape[1]), dtype=np.float64)
    for cx in (0, 1):
        wx = f[0] if cx else 1.0 - f[0]
        ix = (idx[0] + cx) % n_mesh
        for cy in (0, 1):
            wy = f[1] if cy else 1.0 - f[1]
            iy = (idx[1] + cy) % n_mesh
            for cz in (0, 1):
                wz = f[2] if cz else 1.0 - f[2]
                iz = (idx[2] + cz) % n_mesh
                out += wx * wy * wz * flat[:, (ix * n_mesh + iy) * n_mesh + iz]
    return out


def pm_force(pos, n_mesh, box, deconv_power=1):
    """grad(psi) at each particle (shape (3, n)), with lap(psi) = delta: the PM force step of Sec. 2.4."""
    pos = np.asarray(pos)
    C = deposit_fixed(pos, n_mesh, box)
    g = force_mesh(C, pos.shape[1], n_mesh, box, deconv_power)
    return gather(g, pos, n_mesh, box)
