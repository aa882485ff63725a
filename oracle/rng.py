"""Counter-based white noise for the Gaussian initial density field.

Oracle (test infrastructure only). The paper draws its initial field with the 2LPTic generator (Sec. 5), whose random
sequence cannot be reproduced here. Reading taken: one unit Gaussian per lattice point, drawn from the SplitMix64
generator of Steele, Lea & Flood (2014) used in counter mode, and the Box-Muller transform (1958):

    out(c)   = mix(seed + (c + 1) * 0x9E3779B97F4A7C15 mod 2^64), the c-th output of a SplitMix64 stream at `seed`
    u(c)     = ((out(c) >> 11) + 0.5) * 2^-53                      (uniform in (0, 1))
    n(idx)   = sqrt(-2 ln u(2 idx)) * cos(2 pi u(2 idx + 1))       (lattice index idx = (i N + j) N + l)
"""
import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed, counter):
    """The counter-th (0-based) output of a SplitMix64 stream whose state starts at `seed` (uint64 arithmetic)."""
    c = np.asarray(counter, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (c + np.uint64(1)) * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform_open(seed, counter):
    """Uniform doubles in the open interval (0, 1) from the top 53 bits of each output."""
    z = splitmix64(seed, counter)
    return ((z >> np.uint64(11)).astype(np.float64) + 0.5) * 2.0**-53


def white_noise(seed, n_side):
    """Unit-variance Gaussian white noise on the n_side^3 particle lattice, shape (N, N, N), x-major."""
    idx = np.arange(n_side**3, dtype=np.uint64)
    u1 = uniform_open(seed, np.uint64(2) * idx)
    u2 = uniform_open(seed, np.uint64(2) * idx + np.uint64(1))
    g = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
    return g.reshape(n_side, n_side, n_side)
