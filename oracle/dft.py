"""Brute-force discrete Fourier transforms, used only to pin the FFT-based steps of the oracle and the GPU path.

Oracle (test infrastructure only). X(n) = sum_x f(x) exp(-2 pi i n.x / N), written as an explicit O(N^6) sum over all
mesh points (the unnormalised forward convention that both paths use).
"""
import numpy as np


def dft3_brute(f):
    """Full complex 3-D DFT of f (shape (N0, N1, N2)) by direct summation over every point, for every mode."""
    f = np.asarray(f)
    n0, n1, n2 = f.shape
    x0, x1, x2 = np.meshgrid(np.arange(n0), np.arange(n1), np.arange(n2), indexing="ij")
    xs = (x0.ravel(), x1.ravel(), x2.ravel())
    vals = f.ravel().astype(np.complex128)
    out = np.empty((n0, n1, n2), dtype=np.complex128)
    for k0 in range(n0):
        for k1 in range(n1):
            for k2 in range(n2):
                phase = k0 * xs[0] / n0 + k1 * xs[1] / n1 + k2 * xs[2] / n2
                out[k0, k1, k2] = np.sum(vals * np.exp(-2j * np.pi * phase))
    return out


def idft3_brute(F):
    """Unnormalised inverse: f(x) = sum_n F(n) exp(+2 pi i n.x / N), by direct summation."""
    return np.conj(dft3_brute(np.conj(np.asarray(F))))
