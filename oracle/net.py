"""FP64 oracle of the learned displacement correction: a small 3-level 3-D U-Net on the particle lattice.

Test infrastructure only (see oracle/__init__.py). The network is not in the paper: it is the learned part of this
implementation, trained to move a coarse-mesh COLA run (Nm = N, Sec. 2.4 force on a coarse mesh) toward a fine-mesh
run (Nm = 3N). Its definition lives here and in include/lpc.h; this file writes it out plainly.

Tensors are channels-first NumPy arrays (C, D, D, D) on a periodic D^3 grid. Layers:
  conv3(x, W, b)  out[o, p] = b[o] + sum_{i, t} W[o, t, i] x[i, p + t - 1]   (t in {0,1,2}^3, circular)
  down2(x, W, b)  out[o, y] = b[o] + sum_{i, t} W[o, t, i] x[i, 2y + t]      (t in {0,1}^3)
  up2(x, W, b)    out[o, 2y + t] = b[o] + sum_i W[o, t, i] x[i, y]
  leaky(z)        z if z > 0 else 0.1 z
Network (input 6 channels: the coarse run's displacement from the lattice and the first-order 2LPT displacement Psi1,
both in lattice units; output 3 channels: the residual displacement):
  a0 = leaky(conv3(in))            16 @ D
  s0 = leaky(conv3(a0))            16 @ D
  a1 = leaky(down2(s0))            32 @ D/2
  s1 = leaky(conv3(a1))            32 @ D/2
  a2 = leaky(down2(s1))            64 @ D/4
  b2 = leaky(conv3(a2))            64 @ D/4
  u1 = leaky(up2(b2))              32 @ D/2
  c1 = leaky(conv3([u1, s1]))      32 @ D/2
  u0 = leaky(up2(c1))              16 @ D
  c0 = leaky(conv3([u0, s0]))      16 @ D
  out = conv3(c0)                   3 @ D
Loss: mean over voxels and channels of (out - target)^2. Parameters are one flat FP32/FP64 vector: for every layer in
the order above, W as [Cout][taps][Cin] (taps x-major: t = (tx K + ty) K + tz), then b[Cout].
"""
import numpy as np

SLOPE = 0.1
# (name, kind, cin, cout)
LAYERS = (
    ("e0a", "conv3", 6, 16),
    ("e0b", "conv3", 16, 16),
    ("d1", "down2", 16, 32),
    ("e1", "conv3", 32, 32),
    ("d2", "down2", 32, 64),
    ("b2", "conv3", 64, 64),
    ("u1", "up2", 64, 32),
    ("c1", "conv3", 64, 32),
    ("u0", "up2", 32, 16),
    ("c0", "conv3", 32, 16),
    ("out", "conv3", 16, 3),
)
TAPS = {"conv3": 27, "down2": 8, "up2": 8}


def layer_slices():
    """{name: (W slice, b slice, kind, cin, cout)} into the flat parameter vector."""
    out, off = {}, 0
    for name, kind, cin, cout in LAYERS:
        nw = cout * TAPS[kind] * cin
        out[name] = (slice(off, off + nw), slice(off + nw, off + nw + cout), kind, cin, cout)
        off += nw + cout
    return out


def param_count():
    return sum(cout * TAPS[kind] * cin + cout for _, kind, cin, cout in LAYERS)


def unpack(params):
    """{name: (W[Cout][taps][Cin], b[Cout])} views of the flat vector."""
    res = {}
    for name, (ws, bs, kind, cin, cout) in layer_slices().items():
        res[name] = (params[ws].reshape(cout, TAPS[kind], cin), params[bs])
    return res


def taps3():
    return [(tx, ty, tz) for tx in range(3) for ty in range(3) for tz in range(3)]


def taps2():
    return [(tx, ty, tz) for tx in range(2) for ty in range(2) for tz in range(2)]


# --- layers --------------------------------------------------------------------------------------------------------

def conv3(x, W, b):
    cout = W.shape[0]
    out = np.zeros((cout,) + x.shape[1:])
    for t, (tx, ty, tz) in enumerate(taps3()):
        # x[i, p + t - 1] as an array over p
        xs = np.roll(x, shift=(-(tx - 1), -(ty - 1), -(tz - 1)), axis=(1, 2, 3))
        out += np.einsum("oi,ixyz->oxyz", W[:, t, :], xs)
    return out + b[:, None, None, None]


def conv3_backward(x, W, dout):
    """(dx, dW, db) of conv3 given the gradient of its output."""
    dx = np.zeros_like(x)
    dW = np.zeros_like(W)
    for t, (tx, ty, tz) in enumerate(taps3()):
        sh = (-(tx - 1), -(ty - 1), -(tz - 1))
        xs = np.roll(x, shift=sh, axis=(1, 2, 3))
        dW[:, t, :] = np.einsum("oxyz,ixyz->oi", dout, xs)
        # out[p] uses x[p + t - 1]  =>  dx[q] += W^T dout[q - t + 1]
        dx += np.roll(np.einsum("oi,oxyz->ixyz", W[:, t, :], dout), shift=tuple(-s for s in sh), axis=(1, 2, 3))
    return dx, dW, dout.sum(axis=(1, 2, 3))


def down2(x, W, b):
    cout = W.shape[0]
    d = x.shape[1] // 2
    out = np.zeros((cout, d, d, d))
    for t, (tx, ty, tz) in enumerate(taps2()):
        out += np.einsum("oi,ixyz->oxyz", W[:, t, :], x[:, tx::2, ty::2, tz::2])
    return out + b[:, None, None, None]


def down2_backward(x, W, dout):
    dx = np.zeros_like(x)
    dW = np.zeros_like(W)
    for t, (tx, ty, tz) in enumerate(taps2()):
        dW[:, t, :] = np.einsum("oxyz,ixyz->oi", dout, x[:, tx::2, ty::2, tz::2])
        dx[:, tx::2, ty::2, tz::2] = np.einsum("oi,oxyz->ixyz", W[:, t, :], dout)
    return dx, dW, dout.sum(axis=(1, 2, 3))


def up2(x, W, b):
    cout = W.shape[0]
    d = x.shape[1]
    out = np.zeros((cout, 2 * d, 2 * d, 2 * d))
    for t, (tx, ty, tz) in enumerate(taps2()):
        out[:, tx::2, ty::2, tz::2] = np.einsum("oi,ixyz->oxyz", W[:, t, :], x)
    return out + b[:, None, None, None]


def up2_backward(x, W, dout):
    dx = np.zeros_like(x)
    dW = np.zeros_like(W)
    for t, (tx, ty, tz) in enumerate(taps2()):
        g = dout[:, tx::2, ty::2, tz::2]
        dW[:, t, :] = np.einsum("oxyz,ixyz->oi", g, x)
        dx += np.einsum("oi,oxyz->ixyz", W[:, t, :], g)
    return dx, dW, dout.sum(axis=(1, 2, 3))


def leaky(z):
    return np.where(z > 0, z, SLOPE * z)


def leaky_backward(a, da):
    """Gradient through leaky given its output a (the sign of a is the sign of its input)."""
    return np.where(a > 0, da, SLOPE * da)


# --- network -------------------------------------------------------------------------------------------------------

LAYER_FN = {"conv3": conv3, "down2": down2, "up2": up2}
LAYER_BWD = {"conv3": conv3_backward, "down2": down2_backward, "up2": up2_backward}


def forward(params, x):
    """Network output and the cache of every activation."""
    P = unpack(np.asarray(params, dtype=np.float64))
    c = {"in": np.asarray(x, dtype=np.float64)}

    def lay(name, inp, act=True):
        W, b = P[name]
        z = LAYER_FN[layer_slices()[name][2]](inp, W, b)
        return leaky(z) if act else z

    c["a0"] = lay("e0a", c["in"])
    c["s0"] = lay("e0b", c["a0"])
    c["a1"] = lay("d1", c["s0"])
    c["s1"] = lay("e1", c["a1"])
    c["a2"] = lay("d2", c["s1"])
    c["b2"] = lay("b2", c["a2"])
    c["u1"] = lay("u1", c["b2"])
    c["cat1"] = np.concatenate([c["u1"], c["s1"]], axis=0)
    c["c1"] = lay("c1", c["cat1"])
    c["u0"] = lay("u0", c["c1"])
    c["cat0"] = np.concatenate([c["u0"], c["s0"]], axis=0)
    c["c0"] = lay("c0", c["cat0"])
    c["out"] = lay("out", c["c0"], act=False)
    return c["out"], c


def loss(out, target):
    return float(np.mean((out - target) ** 2))


def loss_and_grad(params, x, target):
    """Loss and its gradient with respect to the flat parameter vector (backpropagation through forward)."""
    params = np.asarray(params, dtype=np.float64)
    P = unpack(params)
    out, c = forward(params, x)
    L = loss(out, target)
    grad = np.zeros_like(params)
    sl = layer_slices()

    def back(name, inp, a, da, act=True):
        """Gradient of layer `name` (input inp, output a) given d(loss)/d(a); returns d(loss)/d(inp)."""
        dz = leaky_backward(a, da) if act else da
        W, _ = P[name]
        dx, dW, db = LAYER_BWD[sl[name][2]](inp, W, dz)
        grad[sl[name][0]] = dW.ravel()
        grad[sl[name][1]] = db
        return dx

    dout = 2.0 * (out - target) / out.size
    dc0 = back("out", c["c0"], c["out"], dout, act=False)
    dcat0 = back("c0", c["cat0"], c["c0"], dc0)
    du0, ds0 = dcat0[:16], dcat0[16:].copy()
    dc1 = back("u0", c["c1"], c["u0"], du0)
    dcat1 = back("c1", c["cat1"], c["c1"], dc1)
    du1, ds1 = dcat1[:32], dcat1[32:].copy()
    db2 = back("u1", c["b2"], c["u1"], du1)
    da2 = back("b2", c["a2"], c["b2"], db2)
    ds1 += back("d2", c["s1"], c["a2"], da2)
    da1 = back("e1", c["a1"], c["s1"], ds1)
    ds0 += back("d1", c["s0"], c["a1"], da1)
    da0 = back("e0b", c["a0"], c["s0"], ds0)
    back("e0a", c["in"], c["a0"], da0)
    return L, grad


def adam_step(params, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015) with bias correction; t counts from 1. Returns new (params, m, v)."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mhat = m / (1 - beta1**t)
    vhat = v / (1 - beta2**t)
    return params - lr * mhat / (np.sqrt(vhat) + eps), m, v


# --- features ------------------------------------------------------------------------------------------------------

def input_grid(pos, psi1, ids, n_side, box):
    """Network input (6, N, N, N): the displacement from the lattice (displacement_grid) and Psi1 / (L / N)."""
    dp = box / n_side
    g = np.zeros((3, n_side**3))
    g[:, np.asarray(ids)] = np.asarray(psi1, dtype=np.float64) / dp
    return np.concatenate([displacement_grid(pos, ids, n_side, box), g.reshape(3, n_side, n_side, n_side)])


def displacement_grid(pos, ids, n_side, box, ref=None):
    """Lagrangian displacement field on the lattice, in lattice units, channels-first (3, N, N, N).

    pos[3][n], ids[n] (lattice index (i N + j) N + l, lattice point q = (i + 1/2, j + 1/2, l + 1/2) L / N). With ref
    (positions of the same particles in another run, same order) the field is the minimal-image difference pos - ref
    instead of pos - q."""
    pos = np.asarray(pos, dtype=np.float64)
    ids = np.asarray(ids)
    dp = box / n_side
    if ref is None:
        i, j, l = ids // (n_side * n_side), (ids // n_side) % n_side, ids % n_side
        base = (np.stack([i, j, l]).astype(np.float64) + 0.5) * dp
    else:
        base = np.asarray(ref, dtype=np.float64)
    d = pos - base
    d -= box * np.round(d / box)
    grid = np.zeros((3, n_side**3))
    grid[:, ids] = d / dp
    return grid.reshape(3, n_side, n_side, n_side)


# --- training-data augmentation -------------------------------------------------------------------------------------

# Axis permutations of the cube's symmetries: symmetry k = 8 p + f takes permutation PERMS[p] and reflection bits f
PERMS = ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0))


def cube_symmetry(grid, k):
    """The k-th (0..47) symmetry of the periodic cube applied to a lattice field of 3-vectors, channels-first
    (3 m, N, N, N). The map of space: x'_d = x_{perm[d]}, then for each bit d of f the reflection x'_d -> L - x'_d
    about the box centre, which takes lattice site i (point (i + 1/2) L / N) to N - 1 - i. A vector v at site u goes to
    site T(u) as v'_d = +-v_{perm[d]} (minus for a reflected axis d)."""
    grid = np.asarray(grid)
    perm, f = PERMS[k // 8], k % 8
    n = grid.shape[1]
    out = np.empty_like(grid)
    o = np.indices((n, n, n))                      # output site coordinates o_d
    src = [None] * 3
    for d in range(3):
        src[perm[d]] = (n - 1 - o[d]) if (f >> d) & 1 else o[d]   # input coordinate along axis perm[d]
    for c in range(grid.shape[0]):
        d = c % 3
        sign = -1.0 if (f >> d) & 1 else 1.0
        out[c] = sign * grid[3 * (c // 3) + perm[d]][src[0], src[1], src[2]]
    return out
