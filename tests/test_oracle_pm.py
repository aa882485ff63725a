"""Pins for oracle/pm.py and oracle/dft.py: brute-force DFT, exact fixed-point deposit, sinusoid Poisson solve,
zero net force."""
import numpy as np
import pytest

import synth
from oracle import dft, pm


@pytest.mark.parametrize("shape", [(8, 8, 8), (6, 10, 12), (5, 3, 4)])
def test_numpy_fft_conventions_match_brute_force(shape):
    f = synth.random_real_mesh(7, shape).astype(np.float64)
    F = dft.dft3_brute(f)
    assert np.allclose(np.fft.rfftn(f), F[..., : shape[2] // 2 + 1], rtol=0, atol=1e-10)
    back = dft.idft3_brute(F) / f.size
    assert np.allclose(back.real, f, atol=1e-12)
    assert np.allclose(np.fft.irfftn(np.fft.rfftn(f), s=shape, axes=(0, 1, 2)), f, atol=1e-12)


def test_single_particle_weights_by_hand():
    """A particle at cell (3 + 1/4, 5 + 1/2, 62 + 3/4) of a 64^3 mesh (L = 64): weights (3/4,1/4)x(1/2,1/2)x(1/4,3/4)."""
    one = 1 << 16
    pos = np.array([[3.25], [5.5], [62.75]])
    C = pm.deposit_fixed(pos, 64, 64.0)
    w = {0: (one * 3 // 4, one // 4), 1: (one // 2, one // 2), 2: (one // 4, one * 3 // 4)}
    expected = np.zeros((64, 64, 64), dtype=np.int64)
    for cx in (0, 1):
        for cy in (0, 1):
            for cz in (0, 1):
                expected[3 + cx, 5 + cy, (62 + cz) % 64] = w[0][cx] * w[1][cy] * w[2][cz]
    assert np.array_equal(C, expected)


def test_periodic_wrap_and_box_edge():
    """A particle in the last cell deposits into cell 0; x = L (FP32 rounding of a wrapped value) lands on node 0."""
    C = pm.deposit_fixed(np.array([[63.5], [0.0], [64.0]]), 64, 64.0)
    one = 1 << 16
    assert C[63, 0, 0] == (one // 2) * one * one and C[0, 0, 0] == (one // 2) * one * one
    assert C.sum() == one**3


@pytest.mark.parametrize("seed", [0, 1])
def test_mass_conservation_exact(seed):
    pos = synth.clustered_positions(seed, 5000, 100.0)
    C = pm.deposit_fixed(pos, 32, 100.0)
    assert C.dtype == np.int64 and int(C.sum()) == 5000 * 2**48


def test_lattice_gives_uniform_counts_and_shift_moves_them():
    n = 16
    g = (np.arange(n) * (200.0 / n))
    q = np.array(np.meshgrid(g, g, g, indexing="ij")).reshape(3, -1)
    C = pm.deposit_fixed(q, n, 200.0)
    assert np.all(C == 2**48)
    # a clumpy field shifted by exactly one mesh cell along y shifts C by one index exactly
    pos = synth.clustered_positions(3, 3000, 200.0).astype(np.float64)
    C0 = pm.deposit_fixed(pos, n, 200.0)
    C1 = pm.deposit_fixed(np.mod(pos + np.array([[0.0], [200.0 / n], [0.0]]), 200.0), n, 200.0)
    assert np.array_equal(np.roll(C0, 1, axis=1), C1)


def test_deposit_is_order_independent():
    pos = synth.clustered_positions(4, 4000, 50.0)
    perm = np.random.default_rng(0).permutation(pos.shape[1])
    assert np.array_equal(pm.deposit_fixed(pos, 16, 50.0), pm.deposit_fixed(pos[:, perm], 16, 50.0))


@pytest.mark.parametrize("p", [0, 1, 2])
@pytest.mark.parametrize("m", [(1, 0, 0), (2, -3, 1), (0, 5, 7)])
def test_sinusoid_poisson_closed_form(m, p):
    """delta = A cos(k.x) on the mesh  =>  grad(psi) = A k sin(k.x) / |k|^2 / W(m)^p exactly."""
    n, box, A = 16, 80.0, 0.7
    x = np.arange(n) * (box / n)
    X = np.array(np.meshgrid(x, x, x, indexing="ij"))
    k = 2 * np.pi * np.array(m, dtype=np.float64) / box
    phase = np.tensordot(k, X, axes=1)
    delta = A * np.cos(phase)
    W = np.prod([np.sinc(mi / n) ** 2 for mi in m])
    g = pm.force_mesh_from_delta(delta, box, deconv_power=p)
    for j in range(3):
        expected = A * k[j] * np.sin(phase) / (k @ k) / W**p
        assert np.allclose(g[j], expected, atol=1e-12 * A / np.sqrt(k @ k))


def test_nyquist_derivative_is_zero():
    n, box = 8, 8.0
    x = np.arange(n)
    delta = np.cos(np.pi * x)[:, None, None] * np.ones((1, n, n))  # pure Nyquist mode along x
    g = pm.force_mesh_from_delta(delta, box)
    assert np.abs(g).max() < 1e-14


@pytest.mark.parametrize("p", [0, 2])
def test_zero_net_force(p):
    """sum_p g_p == 0: the gather is the transpose of the deposit and the k = 0 / Nyquist terms vanish."""
    pos = synth.clustered_positions(5, 6000, 120.0).astype(np.float64)
    g = pm.pm_force(pos, 24, 120.0, deconv_power=p)
    scale = np.abs(g).sum(axis=1)
    assert np.all(np.abs(g.sum(axis=1)) < 1e-10 * scale)


def test_unperturbed_lattice_feels_no_force():
    n = 12
    g1 = np.arange(n) * (60.0 / n)
    q = np.array(np.meshgrid(g1, g1, g1, indexing="ij")).reshape(3, -1)
    assert np.abs(pm.pm_force(q, 2 * n, 60.0)).max() < 1e-12


def test_gather_of_linear_ramp_is_exact_inside():
    """CIC interpolation reproduces a field linear in x between nodes (away from the periodic seam)."""
    n, box = 16, 16.0
    field = np.zeros((3, n, n, n))
    field[0] = np.arange(n, dtype=np.float64)[:, None, None]
    pos = np.array([[2.3, 7.75, 13.0], [1.0, 4.5, 9.9], [0.1, 15.2, 8.0]])
    out = pm.gather(field, pos, n, box)
    frac_pos = np.floor(pos[0] * 2**16) / 2**16
    assert np.allclose(out[0], frac_pos, atol=1e-12)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_plane_wave_sampled_force_equals_oracle(axis):
    """The separable lattice input of tests/plane_wave.py, displaced along each axis in turn: its factored counts equal
    deposit_fixed bit for bit, and the mode sum over the density's support equals pm.pm_force (full FFTs) at every
    sampled particle (N = 32, Nm = 96)."""
    from tests import plane_wave as pw
    N, nm = 32, 96
    box = float(nm)
    pos = pw.lattice_plane_wave(N, box, 0.4 * box / N, 3, axis)
    X, Y, Z = pw.factors(pos, N, nm, box)
    C = pm.deposit_fixed(pos.astype(np.float64), nm, box)
    assert np.array_equal(C, X[:, None, None] * Y[None, :, None] * Z[None, None, :])
    sample = np.random.default_rng(5).choice(N**3, 300, replace=False)
    for p in (1, 2):
        ref = pm.pm_force(pos.astype(np.float64), nm, box, deconv_power=p)[:, sample]
        got = pw.force_at(pos, N, nm, box, sample, deconv_power=p)
        assert np.abs(got - ref).max() < 1e-10 * np.abs(ref).max()


def test_fixed_point_overflow_rule():
    """A cell overflows when its exact count reaches 2^63. Particles on a mesh node put their whole 2^48 on one cell:
    32767 of them fit, 32768 reach 2^63 exactly. 70000 wrap a 64-bit sum past 2^64 (the wrapped value has bit 63
    clear), and are still flagged. Particles at a cell centre put 2^45 on each of 8 cells: 2^18 - 1 fit, 2^18 not."""
    nm, box = 16, 50.0
    node = np.full((3, 1), 12.5, dtype=np.float64)                 # 12.5 / (50 / 16) = 4 cells: a node
    centre = np.full((3, 1), 12.5 + 0.5 * box / nm, dtype=np.float64)
    assert not pm.fixed_point_overflow(np.repeat(node, 32767, axis=1), nm, box)
    assert pm.fixed_point_overflow(np.repeat(node, 32768, axis=1), nm, box)
    many = np.repeat(node, 70000, axis=1)
    assert pm.fixed_point_overflow(many, nm, box)
    wrapped = (70000 * 2**48) % 2**64
    assert wrapped < 2**63 and int(pm.deposit_fixed(many, nm, box).max()) == wrapped
    assert not pm.fixed_point_overflow(np.repeat(centre, 2**18 - 1, axis=1), nm, box)
    assert pm.fixed_point_overflow(np.repeat(centre, 2**18, axis=1), nm, box)
    # spread particles never come close
    rng = np.random.default_rng(0)
    assert not pm.fixed_point_overflow(rng.random((3, 10000)) * box, nm, box)
