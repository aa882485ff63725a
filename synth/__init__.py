"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds workload parameters and random-input recipes only. It contains none of the method's arithmetic
(no cosmology, no deposit, no FFT, no integrator), so both the GPU path's tests and the CPU oracle may draw from it.

Workloads (flat LCDM, BBKS spectrum with ns = 0.96, sigma8 = 0.8, Om = 0.31, h = 0.68, 2LPT ICs at z = 9, ten steps
uniform in a from 0.1 to 1.0, modified COLA stepping with nLPT = -2.5, CIC window deconvolved once in the force):
  small  : 32^3 particles, 64^3 mesh, 256 Mpc/h box    (the size the oracle finishes in seconds)
  single : 256^3 particles, 768^3 mesh, 1000 Mpc/h box
  large  : 512^3 particles, 1024^3 mesh, 2000 Mpc/h box
  batch  : 48 boxes, N = {96, 128, 160}[j mod 3], Nm = 2N, L = 300 + 300 j / 47
  learned: coarse (Nm = N) vs fine (Nm = 3N) pairs of 128^3 particles in 500 Mpc/h boxes; applied at 256^3 / 1000
"""
import numpy as np

COSMOLOGY = {"omega_m": 0.31, "h": 0.68, "sigma8": 0.8, "n_s": 0.96}
STEPPING = {"cola": 1, "modified": 1, "n_lpt": -2.5, "deconv_power": 1}
A_LIST = [0.1 + 0.09 * i for i in range(11)]

WORKLOADS = {
    "small": {"n_side": 32, "n_mesh": 64, "box": 256.0, "seed": 1},
    "single": {"n_side": 256, "n_mesh": 768, "box": 1000.0, "seed": 2015},
    "large": {"n_side": 512, "n_mesh": 1024, "box": 2000.0, "seed": 3},
}


def batch_workload():
    """The 48 uneven boxes of the batched form (seeds 1000 + j)."""
    out = []
    for j in range(48):
        n = (96, 128, 160)[j % 3]
        out.append({"n_side": n, "n_mesh": 2 * n, "box": 300.0 + 300.0 * j / 47.0, "seed": 1000 + j})
    return out


def uniform_positions(seed, n, box):
    """n particles uniform in [0, box)^3, float32, shape (3, n)."""
    rng = np.random.default_rng(seed)
    return (rng.random((3, n)) * box).astype(np.float32)


def clustered_positions(seed, n, box, n_clumps=8, sigma_frac=0.01, frac_in_clumps=0.7):
    """A clumpy distribution: a fraction of the particles in tight Gaussian clumps (late-time halo-like cells)."""
    rng = np.random.default_rng(seed)
    n_in = int(n * frac_in_clumps)
    centres = rng.random((3, n_clumps)) * box
    which = rng.integers(0, n_clumps, size=n_in)
    clumped = centres[:, which] + rng.normal(0.0, sigma_frac * box, size=(3, n_in))
    rest = rng.random((3, n - n_in)) * box
    pos = np.concatenate([clumped, rest], axis=1) % box
    return pos.astype(np.float32)


def edge_positions(n_mesh, box):
    """Positions on cell boundaries, at the box edge and just below it (float32), shape (3, m)."""
    cell = box / n_mesh
    vals = np.array([0.0, cell, 0.5 * cell, box - cell, np.nextafter(np.float32(box), np.float32(0)),
                     np.float32(box) * (1 - 2**-24)], dtype=np.float32)
    g = np.array(np.meshgrid(vals, vals, vals, indexing="ij")).reshape(3, -1)
    return g.astype(np.float32)


def random_real_mesh(seed, shape):
    """Standard-normal float32 real mesh (FFT parity inputs)."""
    return np.random.default_rng(seed).standard_normal(shape).astype(np.float32)
