"""FP64 oracle of the reduced bispectrum Q(k1, k2, k3) of a periodic density field (Sec. 7: the paper compares the
reduced bispectrum of its runs with N-body runs). Test infrastructure only (see oracle/__init__.py).

Estimator (the paper gives the definition, not an estimator): with delta_hat the unnormalised DFT of the density
contrast on an Nm^3 mesh (continuous delta(k) = V/M delta_hat, M = Nm^3, V = L^3), and shells b = {n : |k_n| in
[k_b - dk/2, k_b + dk/2)},
    B(k1, k2, k3) = V^2 / M^3 * sum over triangles n1 + n2 + n3 = 0 (n_i in shell i) of delta_hat1 delta_hat2
                    delta_hat3, divided by the number of such triangles,
    P(k_b)        = V / M^2 * mean over shell b of |delta_hat|^2,
    Q             = B / (P1 P2 + P2 P3 + P3 P1).
The triangle sum is evaluated with inverse FFTs of the shell-filtered fields (sum over x of the product of the three
filtered fields, over the same product for the shell indicators); bispectrum_brute() sums the triangles directly.
"""
import numpy as np


def wavenumbers(nm, box):
    """|k| (h/Mpc) of every mode of the full nm^3 FFT grid."""
    n = np.fft.fftfreq(nm, d=1.0 / nm)
    kf = 2 * np.pi / box
    kx, ky, kz = np.meshgrid(n, n, n, indexing="ij")
    return kf * np.sqrt(kx**2 + ky**2 + kz**2)


def shell(kmag, kc, dk):
    return (kmag >= kc - 0.5 * dk) & (kmag < kc + 0.5 * dk)


def power_in_shell(dhat, box, kc, dk):
    nm = dhat.shape[0]
    M = nm**3
    s = shell(wavenumbers(nm, box), kc, dk)
    return box**3 / M**2 * float(np.mean(np.abs(dhat[s]) ** 2))


def bispectrum(dhat, box, k1, k2, k3, dk):
    """(B, Q) from the full complex delta_hat (nm^3) with the FFT shell estimator."""
    nm = dhat.shape[0]
    M = nm**3
    kmag = wavenumbers(nm, box)
    fields, ind = [], []
    for kc in (k1, k2, k3):
        s = shell(kmag, kc, dk)
        fields.append(np.fft.ifftn(np.where(s, dhat, 0.0)).real * M)      # sum_{n in shell} dhat e^{ikx}
        ind.append(np.fft.ifftn(s.astype(np.float64)).real * M)           # number-of-modes kernel
    num = float(np.sum(fields[0] * fields[1] * fields[2]))
    den = float(np.sum(ind[0] * ind[1] * ind[2]))
    B = box**6 / M**3 * num / den
    p = [power_in_shell(dhat, box, kc, dk) for kc in (k1, k2, k3)]
    Q = B / (p[0] * p[1] + p[1] * p[2] + p[2] * p[0])
    return B, Q


def bispectrum_brute(dhat, box, k1, k2, k3, dk):
    """B by summing every triangle n1 + n2 + n3 = 0 with n_i in shell i (small meshes only)."""
    nm = dhat.shape[0]
    M = nm**3
    kmag = wavenumbers(nm, box)
    idx = [np.argwhere(shell(kmag, kc, dk)) for kc in (k1, k2, k3)]
    s3 = shell(kmag, k3, dk)
    total, count = 0.0, 0
    for a in idx[0]:
        for b in idx[1]:
            c = (-(a + b)) % nm
            if s3[c[0], c[1], c[2]]:
                total += (dhat[tuple(a)] * dhat[tuple(b)] * dhat[tuple(c)]).real
                count += 1
    return box**6 / M**3 * total / count


def delta_hat_from_particles(pos, nm, box, deconvolve=True):
    """Full complex DFT of the CIC density contrast of particles pos[3][n] (the oracle's fixed-point deposit),
    divided once by the CIC window when deconvolve is set."""
    from oracle import pm
    pos = np.asarray(pos)
    C = pm.deposit_fixed(pos, nm, box)
    delta = C.astype(np.float64) * (nm**3 / pos.shape[1]) * 2.0**-48 - 1.0
    dhat = np.fft.fftn(delta)
    if deconvolve:
        n = np.fft.fftfreq(nm, d=1.0 / nm)
        w1 = np.sinc(n / nm) ** 2
        dhat = dhat / (w1[:, None, None] * w1[None, :, None] * w1[None, None, :])
    return dhat
