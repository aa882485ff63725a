"""Sampled evaluation of the oracle's PM force (oracle/pm.py) for a lattice displaced along one axis only.

Test infrastructure: it applies the oracle's own definitions (fixed-point CIC deposit, CIC window W^p, Green's function
-1/k^2, spectral derivative i k_j, Nyquist and k = 0 zeroing, 1/Nm^3 inverse normalisation, fixed-point CIC gather)
to a special input on which they can be evaluated particle by particle at full size.

The input: N^3 particles at lattice cell centres q = (i + 1/2) L / N, displaced along one axis (x unless stated) by a
function of that axis's q, in a box with L = Nm (so the fixed-point scale Nm 2^16 / L is 2^16 and every undisplaced
coordinate, 3 j + 3/2 for Nm = 3 N, is exact). A particle's deposit weights are a product of per-axis weights, and its
x weights depend on i alone, its y weights on j alone, its z weights on l alone, so the counts factor exactly:
C = X (x) Y (x) Z with X, Y, Z the summed per-axis weights of one lattice line. The two undisplaced factors repeat
with the lattice period, so their DFTs vanish except at multiples of N: the density spectrum, and with it each
gradient spectrum, lives on Nm x (few) x (few) modes (the displaced axis taking all Nm), and the force mesh at any
node is a direct sum over those modes.
"""
import numpy as np

from oracle import pm


def lattice_plane_wave(N, box, amp, mode, axis=0):
    """FP32 positions (3, N^3) in lattice order (i, j, l): coordinate `axis` is q + amp sin(2 pi mode q / L) of its own
    lattice index, the other two are q."""
    q = (np.arange(N, dtype=np.float64) + 0.5) * (box / N)
    qd = q + amp * np.sin(2.0 * np.pi * mode * q / box)
    idx = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
    pos = np.stack([(qd if a == axis else q)[idx[a].ravel()] for a in range(3)]).astype(np.float32)
    return pos


def axis_counts(coord, n_mesh, box):
    """Summed fixed-point CIC weights of 1-D coordinates on one axis (int64, length Nm), as in pm.deposit_fixed."""
    c = np.asarray(coord, dtype=np.float64)
    idx, frac = pm.fixed_point_coords(np.stack([c, c, c]), n_mesh, box)
    one = np.int64(1) << np.int64(pm.FRAC_BITS)
    out = np.zeros(n_mesh, dtype=np.int64)
    np.add.at(out, idx[0], one - frac[0])
    np.add.at(out, (idx[0] + 1) % n_mesh, frac[0])
    return out


def factors(pos, N, n_mesh, box):
    """X, Y, Z with deposit_fixed(pos) == X[:, None, None] * Y[None, :, None] * Z[None, None, :]."""
    p = np.asarray(pos, dtype=np.float64).reshape(3, N, N, N)
    # the construction: x depends on i only, y on j only, z on l only
    assert np.all(p[0] == p[0][:, :1, :1]) and np.all(p[1] == p[1][:1, :, :1]) and np.all(p[2] == p[2][:1, :1, :])
    return (axis_counts(p[0][:, 0, 0], n_mesh, box), axis_counts(p[1][0, :, 0], n_mesh, box),
            axis_counts(p[2][0, 0, :], n_mesh, box))


def force_at(pos, N, n_mesh, box, sample, deconv_power=1):
    """grad(psi) at the particles `sample` (indices into pos), shape (3, len(sample)): pm.pm_force's value there."""
    X, Y, Z = factors(pos, N, n_mesh, box)
    n = N**3
    m = n_mesh**3 / float(n)
    hats = [np.fft.fft(a.astype(np.float64)) for a in (X, Y, Z)]
    # the displaced axis keeps all Nm modes; the two lattice-periodic factors have a few
    sparse = [np.flatnonzero(np.abs(h) > 1e-9 * np.abs(h).max()) for h in hats]
    full = int(np.argmax([len(s) for s in sparse]))
    supp = [np.arange(n_mesh) if a == full else sparse[a] for a in range(3)]
    assert all(len(supp[a]) <= 8 for a in range(3) if a != full), "two factors are not lattice-periodic"
    nf = np.fft.fftfreq(n_mesh, d=1.0 / n_mesh)  # signed mode numbers
    kx, ky, kz = np.meshgrid(nf[supp[0]], nf[supp[1]], nf[supp[2]], indexing="ij")
    # full-spectrum density contrast on the support: (m 2^-3F) X^ Y^ Z^ - Nm^3 [k = 0]
    dh = (m * 2.0 ** (-3 * pm.FRAC_BITS)) * (hats[0][supp[0]][:, None, None] * hats[1][supp[1]][None, :, None] *
                                              hats[2][supp[2]][None, None, :])
    zero = (kx == 0) & (ky == 0) & (kz == 0)
    dh = np.where(zero, dh - n_mesh**3, dh)
    kf = 2.0 * np.pi / box
    k2 = kf**2 * (kx**2 + ky**2 + kz**2)
    W = (np.sinc(kx / n_mesh) * np.sinc(ky / n_mesh) * np.sinc(kz / n_mesh)) ** 2
    base = np.where(zero, 0.0, -1.0 / np.where(zero, 1.0, k2)) / W**deconv_power * dh
    half = n_mesh // 2
    spectra = []
    for kj in (kx, ky, kz):
        spectra.append(np.where(np.abs(kj) == half, 0.0, 1j * kf * kj * base).ravel())
    modes = np.stack([kx.ravel(), ky.ravel(), kz.ravel()])  # (3, K)
    # CIC gather of the force mesh at the sampled particles; mesh nodes by direct inverse sums over the support
    idx, frac = pm.fixed_point_coords(np.asarray(pos, dtype=np.float64)[:, sample], n_mesh, box)
    f = frac.astype(np.float64) * 2.0**-pm.FRAC_BITS
    out = np.zeros((3, len(sample)))
    for cx in (0, 1):
        for cy in (0, 1):
            for cz in (0, 1):
                w = (f[0] if cx else 1.0 - f[0]) * (f[1] if cy else 1.0 - f[1]) * (f[2] if cz else 1.0 - f[2])
                node = np.stack([(idx[0] + cx) % n_mesh, (idx[1] + cy) % n_mesh, (idx[2] + cz) % n_mesh])
                phase = np.exp(2j * np.pi * (node.T.astype(np.float64) @ modes) / n_mesh)  # (S, K)
                for j in range(3):
                    out[j] += w * (phase @ spectra[j]).real / n_mesh**3
    return out
