"""Pins of the learned-correction oracle (oracle/net.py) and of the reduced-bispectrum oracle (oracle/bispectrum.py).

conv3 against scipy.ndimage.correlate (an independent library routine); down2/up2 and conv3 against their adjoint
identities; the whole network's backpropagation against central finite differences; Adam against its closed-form first
step; the displacement features against hand-built lattices; the FFT bispectrum estimator against the brute-force
triangle sum and against the closed form of three plane waves closing a triangle.
"""
import numpy as np
import pytest
from scipy import ndimage

from oracle import bispectrum as obs
from oracle import net


def rand(seed, *shape):
    return np.random.default_rng(seed).standard_normal(shape)


def test_param_count_and_layout():
    # 3-level U-Net of the header: 16/32/64 channels
    want = (16 * 27 * 6 + 16) + (16 * 27 * 16 + 16) + (32 * 8 * 16 + 32) + (32 * 27 * 32 + 32) + (64 * 8 * 32 + 64) \
        + (64 * 27 * 64 + 64) + (32 * 8 * 64 + 32) + (32 * 27 * 64 + 32) + (16 * 8 * 32 + 16) + (16 * 27 * 32 + 16) \
        + (3 * 27 * 16 + 3)
    assert net.param_count() == want
    sl = net.layer_slices()
    assert sl["out"][1].stop == want


def test_conv3_matches_scipy_correlate_wrap():
    x = rand(1, 3, 6, 6, 6)
    W = rand(2, 4, 27, 3)
    b = rand(3, 4)
    got = net.conv3(x, W, b)
    for o in range(4):
        ref = np.full(x.shape[1:], b[o])
        for i in range(3):
            K = W[o, :, i].reshape(3, 3, 3)      # taps x-major
            ref += ndimage.correlate(x[i], K, mode="wrap")
        assert np.allclose(got[o], ref, atol=1e-12)


def test_adjoint_identities():
    x = rand(4, 5, 8, 8, 8)
    W3 = rand(5, 6, 27, 5)
    y3 = rand(6, 6, 8, 8, 8)
    dx, _, _ = net.conv3_backward(x, W3, y3)
    lhs = np.sum(net.conv3(x, W3, np.zeros(6)) * y3)
    assert np.isclose(lhs, np.sum(x * dx), rtol=1e-12)
    W2 = rand(7, 6, 8, 5)
    y2 = rand(8, 6, 4, 4, 4)
    ddx, _, _ = net.down2_backward(x, W2, y2)
    assert np.isclose(np.sum(net.down2(x, W2, np.zeros(6)) * y2), np.sum(x * ddx), rtol=1e-12)
    # up2 with the transposed weights is the adjoint of down2
    Wt = np.transpose(W2, (2, 1, 0))
    assert np.allclose(net.up2(y2, Wt, np.zeros(5)), ddx, atol=1e-12)
    # up2's own backward is consistent with its forward
    dxu, _, _ = net.up2_backward(y2, Wt, x)
    assert np.isclose(np.sum(net.up2(y2, Wt, np.zeros(5)) * x), np.sum(y2 * dxu), rtol=1e-12)


def test_down2_up2_by_hand():
    x = np.zeros((1, 4, 4, 4))
    x[0, 3, 2, 1] = 2.0                       # voxel (3,2,1) = 2 y + t with y = (1,1,0), t = (1,0,1)
    W = np.zeros((1, 8, 1))
    t = (1 * 2 + 0) * 2 + 1
    W[0, t, 0] = 0.5
    out = net.down2(x, W, np.array([0.25]))
    assert out[0, 1, 1, 0] == 1.25 and np.count_nonzero(out - 0.25) == 1
    up = net.up2(out - 0.25, W, np.zeros(1))
    assert up[0, 3, 2, 1] == 0.5 and np.count_nonzero(up) == 1


def test_network_gradient_matches_finite_differences():
    P = net.param_count()
    rng = np.random.default_rng(5)
    params = np.zeros(P)
    for name, (ws, bs, kind, cin, cout) in net.layer_slices().items():
        fan_in = net.TAPS[kind] * cin
        params[ws] = rng.uniform(-1, 1, ws.stop - ws.start) * np.sqrt(6.0 / fan_in)
        params[bs] = rng.uniform(-0.1, 0.1, cout)
    x = rand(6, 6, 8, 8, 8)
    target = rand(7, 3, 8, 8, 8) * 0.5
    L, g = net.loss_and_grad(params, x, target)
    assert np.isclose(L, net.loss(net.forward(params, x)[0], target))
    idx = []
    for name, (ws, bs, kind, cin, cout) in net.layer_slices().items():
        idx += list(rng.integers(ws.start, ws.stop, 3)) + [bs.start]
    h = 1e-6
    for i in idx:
        e = np.zeros(P)
        e[i] = h
        fd = (net.loss(net.forward(params + e, x)[0], target) - net.loss(net.forward(params - e, x)[0], target)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g).max()) + 1e-5 * abs(g[i]), (i, fd, g[i])


def test_adam_first_step_closed_form():
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    p, m, v = net.adam_step(np.ones(4), g, np.zeros(4), np.zeros(4), 1, 0.01)
    # after one step mhat = g and vhat = g^2, so the update is -lr g / (|g| + eps)
    assert np.allclose(p, 1.0 - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_displacement_grid_features():
    n, box = 4, 100.0
    dp = box / n
    ids = np.arange(n**3)
    i, j, l = ids // 16, (ids // 4) % 4, ids % 4
    q = (np.stack([i, j, l]) + 0.5) * dp
    assert np.all(net.displacement_grid(q, ids, n, box) == 0.0)
    pos = q.copy()
    pos[0] += 0.25 * dp
    pos[1] -= 0.75 * dp
    pos %= box
    g = net.displacement_grid(pos, ids, n, box)
    assert np.allclose(g[0], 0.25) and np.allclose(g[1], -0.75) and np.allclose(g[2], 0.0)
    perm = np.random.default_rng(1).permutation(n**3)
    assert np.allclose(net.displacement_grid(pos[:, perm], ids[perm], n, box), g)
    ref = (pos + 0.1 * dp) % box
    assert np.allclose(net.displacement_grid(pos, ids, n, box, ref=ref), -0.1)
    psi1 = np.stack([np.full(n**3, 2.0 * dp), np.zeros(n**3), -0.5 * dp * np.ones(n**3)])
    inp = net.input_grid(pos[:, perm], psi1[:, perm], ids[perm], n, box)
    assert inp.shape == (6, n, n, n)
    assert np.allclose(inp[:3], g) and np.allclose(inp[3], 2.0) and np.allclose(inp[5], -0.5)


def test_bispectrum_fft_estimator_equals_brute_force():
    nm, box = 16, 100.0
    kf = 2 * np.pi / box
    dhat = np.fft.fftn(rand(11, nm, nm, nm) + 0.3 * rand(12, nm, nm, nm) ** 2)
    for k1, k2, k3 in [(3, 3, 3), (2, 4, 5), (4, 4, 6)]:
        B, _ = obs.bispectrum(dhat, box, k1 * kf, k2 * kf, k3 * kf, 1.0 * kf)
        Bb = obs.bispectrum_brute(dhat, box, k1 * kf, k2 * kf, k3 * kf, 1.0 * kf)
        assert np.isclose(B, Bb, rtol=1e-9)


def test_bispectrum_of_three_plane_waves_closed_form():
    """delta = A [cos(k1.x) + cos(k2.x) + cos(k3.x)] with k1 + k2 + k3 = 0 (a 3-4-5 triangle of fundamental modes):
    only the triangles (k1, k2, k3) and (-k1, -k2, -k3) carry amplitude, each (M A / 2)^3, so
    B = V^2 A^3 / (4 N_tri) and P(shell j) = V A^2 / (2 N_j), with N_tri and N_j counted by enumerating the mesh."""
    nm, box, A = 16, 100.0, 0.7
    kf = 2 * np.pi / box
    x = np.arange(nm)
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    ph = 2 * np.pi / nm
    d = A * (np.cos(ph * 3 * X) + np.cos(ph * 4 * Y) + np.cos(ph * (-3 * X - 4 * Y)))
    dhat = np.fft.fftn(d)
    V, M = box**3, nm**3
    # shells of width kf around 3, 4, 5 kf; count their modes and index triangles by enumeration
    n = np.fft.fftfreq(nm, d=1.0 / nm)
    modes = [(a, b, c) for a in n for b in n for c in n]
    def in_shell(m, kc):
        r = np.sqrt(m[0] ** 2 + m[1] ** 2 + m[2] ** 2)
        return kc - 0.5 <= r < kc + 0.5
    sh = {kc: [m for m in modes if in_shell(m, kc)] for kc in (3, 4, 5)}
    s5 = set(sh[5])
    def wrap(v):
        return ((v + nm // 2) % nm) - nm // 2
    n_tri = sum(1 for a in sh[3] for b in sh[4]
                if (wrap(-(a[0] + b[0])), wrap(-(a[1] + b[1])), wrap(-(a[2] + b[2]))) in s5)
    B, Q = obs.bispectrum(dhat, box, 3 * kf, 4 * kf, 5 * kf, kf)
    assert np.isclose(B, V**2 * A**3 / (4 * n_tri), rtol=1e-9)
    P = [V * A**2 / (2 * len(sh[kc])) for kc in (3, 4, 5)]
    assert np.isclose(obs.power_in_shell(dhat, box, 3 * kf, kf), P[0], rtol=1e-9)
    assert np.isclose(Q, B / (P[0] * P[1] + P[1] * P[2] + P[2] * P[0]), rtol=1e-9)


def _transform_points(x, k, box):
    """The cube symmetry k as a map of positions x[3][n] (independent of cube_symmetry's index arithmetic)."""
    perm, f = net.PERMS[k // 8], k % 8
    y = np.stack([x[perm[d]] for d in range(3)])
    for d in range(3):
        if (f >> d) & 1:
            y[d] = box - y[d]
    return y


def test_cube_symmetry_is_the_geometric_map():
    """Moving the particles by symmetry k (positions and the lattice points their ids name, recomputed from scratch)
    and taking their displacement field equals cube_symmetry of the original displacement field, for all 48 k; the
    map is a group action: k = 0 is the identity and the 48 images of a generic field are distinct."""
    n_side, box = 6, 60.0
    dp = box / n_side
    rng = np.random.default_rng(5)
    ids = np.arange(n_side**3)
    ijk = np.stack([ids // (n_side * n_side), (ids // n_side) % n_side, ids % n_side]).astype(np.float64)
    q = (ijk + 0.5) * dp
    x = q + rng.uniform(-0.4, 0.4, q.shape) * dp
    psi = rng.standard_normal(q.shape) * dp
    grid = net.input_grid(x, psi, ids, n_side, box)
    seen = set()
    for k in range(48):
        xt, qt, pt = _transform_points(x, k, box), _transform_points(q, k, box), _transform_points(psi + box, k, box)
        # psi is a vector: transform it as a difference of two points so that reflections flip its sign
        pt = pt - _transform_points(np.full_like(psi, box), k, box)
        t_ijk = np.rint(qt / dp - 0.5).astype(np.int64)
        t_ids = (t_ijk[0] * n_side + t_ijk[1]) * n_side + t_ijk[2]
        assert np.array_equal(np.sort(t_ids), ids)  # the lattice maps onto itself
        ref = net.input_grid(xt % box, pt, t_ids, n_side, box)
        got = net.cube_symmetry(grid, k)
        assert np.allclose(got, ref, rtol=0, atol=1e-12), k
        seen.add(got.tobytes())
    assert np.array_equal(net.cube_symmetry(grid, 0), grid)
    assert len(seen) == 48
