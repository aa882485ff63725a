"""GPU parity of the learned correction (lpc_net_*) against the FP64 oracle in oracle/net.py.

Bars (derived from the precision stated in include/lpc.h): activations, their gradients and the MFMA operands are
BF16 (relative rounding 2^-9 ~ 2e-3 per value). Eleven layers each round their weights and outputs once, so the
network output carries ~ sqrt(22) x 2e-3 ~ 1e-2 relative error: the bar is 3e-2 (relative L2 over the grid). The
parameter gradient passes through the same roundings twice (forward activations, BF16 gradients): bar 6e-2
relative L2 over the whole vector and 1.5e-1 for each layer's block. Adam is FP32 element-wise: 1e-5 relative.
"""
import numpy as np
import pytest

from oracle import net as onet
from tests.gpu_util import rel_l2, requires_gpu, say, to_dev, to_np, torch

pytestmark = [pytest.mark.gpu, requires_gpu]


def grid_to_cf(a, D):
    """GPU channels-last [V][C] -> oracle channels-first (C, D, D, D)."""
    a = np.asarray(a, dtype=np.float64)
    return a.reshape(D, D, D, a.shape[-1]).transpose(3, 0, 1, 2)


def cf_to_grid(a):
    a = np.asarray(a)
    return np.ascontiguousarray(a.transpose(1, 2, 3, 0).reshape(-1, a.shape[0])).astype(np.float32)


def sample(D, seed):
    rng = np.random.default_rng(seed)
    feat = (0.5 * rng.standard_normal((6, D, D, D))).astype(np.float32)
    target = (0.1 * rng.standard_normal((3, D, D, D))).astype(np.float32)
    return feat, target


@pytest.mark.parametrize("D", [8, 16])
def test_forward_matches_oracle(D):
    from paper_1506_03737_amd import lpc
    say(f"net: forward D={D}")
    params = lpc.lpc_net_init(11)
    params[onet.layer_slices()["out"][0]] *= 10.0     # a full-size last layer, so the output is not tiny
    feat, _ = sample(D, 1)
    ws = lpc.net_workspace(D)
    out = torch.empty((D**3, 3), dtype=torch.float32, device="cuda")
    lpc.lpc_net_forward(D, to_dev(params), to_dev(cf_to_grid(feat)), out, ws)  # feat: 6 channels
    ref, _ = onet.forward(params.astype(np.float64), feat.astype(np.float64))
    err = rel_l2(grid_to_cf(to_np(out), D), ref)
    say(f"  rel L2 = {err:.3e}")
    assert err < 3e-2


# D = 8, 16: every weight gradient on the vector-ALU kernels; D = 32, 64: the 3^3 layers on grids of 32 and 64 per
# side take the MFMA weight-gradient kernel (bricks of 4 x 4 x 32; at D = 64 the (cin, cout) pairs (8, 16), (16, 16),
# (32, 16), (16, 3), (32, 32) and (64, 32); the 64 x 64 layer is at D / 4 = 16 and stays on the vector ALUs)
@pytest.mark.parametrize("D", [8, 16, 32, 64])
def test_gradient_matches_oracle(D):
    from paper_1506_03737_amd import lpc
    say(f"net: loss and gradient D={D}")
    params = lpc.lpc_net_init(12)
    params[onet.layer_slices()["out"][0]] *= 10.0
    feat, target = sample(D, 2)
    ws = lpc.net_workspace(D)
    grad = torch.empty(params.size, dtype=torch.float32, device="cuda")
    pd = to_dev(params)
    loss = lpc.lpc_net_loss_grad(D, pd, to_dev(cf_to_grid(feat)), to_dev(cf_to_grid(target)), grad, ws)
    L, g = onet.loss_and_grad(params.astype(np.float64), feat.astype(np.float64), target.astype(np.float64))
    gg = to_np(grad).astype(np.float64)
    say(f"  loss {loss:.6e} vs {L:.6e}; grad rel L2 {rel_l2(gg, g):.3e}")
    assert abs(loss - L) < 3e-2 * L
    assert rel_l2(gg, g) < 6e-2
    for name, (ws_, bs, kind, cin, cout) in onet.layer_slices().items():
        e = rel_l2(gg[ws_], g[ws_])
        eb = rel_l2(gg[bs], g[bs])
        say(f"  {name:4s} W {e:.3e} b {eb:.3e}")
        assert e < 1.5e-1 and eb < 1.5e-1, name
    # deterministic: a second call gives the same bits
    grad2 = torch.empty_like(grad)
    loss2 = lpc.lpc_net_loss_grad(D, pd, to_dev(cf_to_grid(feat)), to_dev(cf_to_grid(target)), grad2, ws)
    assert loss2 == loss and torch.equal(grad, grad2)


def test_adam_matches_oracle():
    from paper_1506_03737_amd import lpc
    say("net: adam")
    P = lpc.lpc_net_param_count()
    rng = np.random.default_rng(3)
    p = rng.standard_normal(P).astype(np.float32)
    m = np.zeros(P, dtype=np.float32)
    v = np.zeros(P, dtype=np.float32)
    pd, md, vd = to_dev(p), to_dev(m), to_dev(v)
    pr, mr, vr = p.astype(np.float64), m.astype(np.float64), v.astype(np.float64)
    for t in range(1, 4):
        g = (rng.standard_normal(P) * 10.0**rng.uniform(-4, 0, P)).astype(np.float32)
        lpc.lpc_net_adam(pd, md, vd, to_dev(g), t, 1e-3)
        pr, mr, vr = onet.adam_step(pr, g.astype(np.float64), mr, vr, t, 1e-3)
    # FP32 rounding of each update term (~6e-8 of its size; m and v can cancel to far below their terms)
    assert np.allclose(to_np(pd), pr, rtol=1e-6, atol=1e-8)
    assert np.allclose(to_np(md), mr, rtol=1e-5, atol=1e-6 * np.abs(mr).max())
    assert np.allclose(to_np(vd), vr, rtol=1e-5, atol=1e-6 * np.abs(vr).max())


def test_features_and_apply():
    from paper_1506_03737_amd import lpc
    say("net: features and apply")
    N, box = 16, 200.0
    dp = box / N
    ids = np.arange(N**3, dtype=np.int32)
    i, j, l = ids // (N * N), (ids // N) % N, ids % N
    q = (np.stack([i, j, l]) + 0.5) * dp
    rng = np.random.default_rng(4)
    pos = ((q + rng.normal(0, 1.5 * dp, q.shape)) % box).astype(np.float32)
    perm = rng.permutation(N**3)
    pos_p, ids_p = np.ascontiguousarray(pos[:, perm]), np.ascontiguousarray(ids[perm])
    ref = ((pos_p + rng.normal(0, 0.3 * dp, pos_p.shape)) % box).astype(np.float32)
    geom = lpc.geometry(N, N, box)
    ws = lpc.net_workspace(N)
    feat = torch.empty((N**3, 3), dtype=torch.float32, device="cuda")
    lpc.lpc_net_features(geom, to_dev(pos_p), to_dev(ids_p), feat, ws)
    want = onet.displacement_grid(pos_p, ids_p, N, box)
    assert np.abs(grid_to_cf(to_np(feat), N) - want).max() < 1e-5
    tgt = torch.empty_like(feat)
    lpc.lpc_net_features(geom, to_dev(pos_p), to_dev(ids_p), tgt, ws, ref_pos=to_dev(ref))
    assert np.abs(grid_to_cf(to_np(tgt), N) - onet.displacement_grid(pos_p, ids_p, N, box, ref=ref)).max() < 1e-5
    # the 6-channel input grid: displacement and Psi1 / dp
    psi1 = rng.normal(0, 2.0 * dp, pos_p.shape).astype(np.float32)
    inp = torch.empty((N**3, 6), dtype=torch.float32, device="cuda")
    lpc.lpc_net_features(geom, to_dev(pos_p), to_dev(ids_p), inp, ws, psi1=to_dev(psi1))
    assert np.abs(grid_to_cf(to_np(inp), N) - onet.input_grid(pos_p, psi1, ids_p, N, box)).max() < 1e-5
    # apply = input grid -> forward -> pos += r dp
    params = lpc.lpc_net_init(5)
    params[onet.layer_slices()["out"][0]] *= 10.0
    pd = to_dev(params)
    out = torch.empty_like(feat)
    lpc.lpc_net_forward(N, pd, inp, out, ws)
    ps = lpc.ParticleSet(to_dev(pos_p), None, to_dev(psi1), None, to_dev(ids_p))
    lpc.lpc_net_apply(geom, pd, ps, ws)
    r = to_np(out)[ids_p].T
    expect = (pos_p.astype(np.float64) + r * dp) % box
    d = to_np(ps.pos) - expect
    d -= box * np.round(d / box)
    assert np.abs(d).max() < 1e-4
    bad = to_dev(np.full(N**3, N**3, dtype=np.int32))
    with pytest.raises(lpc.LpcError):
        lpc.lpc_net_features(geom, to_dev(pos_p), bad, feat, ws)


def test_training_reduces_loss():
    """A hundred Adam steps on one fixed sample (the learnable target: a smooth function of the features) halve the
    loss."""
    from paper_1506_03737_amd import lpc
    say("net: training on one sample")
    D = 16
    feat, _ = sample(D, 6)
    target = (0.3 * np.tanh(feat[:3]) - 0.1 * np.roll(feat[3:], 1, axis=1)).astype(np.float32)
    params = to_dev(lpc.lpc_net_init(9))
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    grad = torch.empty_like(params)
    ws = lpc.net_workspace(D)
    fd, td = to_dev(cf_to_grid(feat)), to_dev(cf_to_grid(target))
    losses = []
    for t in range(1, 101):
        losses.append(lpc.lpc_net_loss_grad(D, params, fd, td, grad, ws))
        lpc.lpc_net_adam(params, m, v, grad, t, 3e-3)
    say(f"  loss {losses[0]:.4e} -> {losses[-1]:.4e}")
    assert losses[-1] < 0.5 * losses[0]
