"""GPU parity of the reduced bispectrum (lpc_bispectrum) against the FP64 oracle (oracle/bispectrum.py), whose
estimator is pinned by brute-force triangle sums and by three plane waves closing a triangle.

The deposit is bitwise the oracle's, so both sides start from the same density; they differ by the FP32 forward and
inverse transforms (relative rounding ~1e-7 per value, growing as log2 of the mesh) and by FP32 storage of the
filtered fields. Shell membership is decided by the same FP64 arithmetic on both sides, so the mode sets agree
exactly. Bars: B, Q and the shell powers within 1.5e-6 relative (measured at most 4.0e-7 on these inputs), at
estimator meshes 48, 64 and 128 (the learned form's evaluation mesh); shells that close no triangle give NaN.
"""
import numpy as np
import pytest

import synth
from oracle import bispectrum as obs
from tests.gpu_util import requires_gpu, say, to_dev

pytestmark = [pytest.mark.gpu, requires_gpu]

TRIANGLES = [(0.05, 0.05, 0.05), (0.1, 0.1, 0.1), (0.2, 0.2, 0.2), (0.1, 0.2, 0.15), (0.1, 0.2, 0.25),
             (0.05, 0.1, 0.12)]
REL = 1.5e-6


@pytest.mark.parametrize("nm,box,n", [(48, 400.0, 30011), (64, 500.0, 120001), (128, 1000.0, 400003)])
def test_bispectrum_matches_oracle(nm, box, n):
    from paper_1506_03737_amd import lpc
    pos = synth.clustered_positions(nm, n, box)
    dk = 3 * 2 * np.pi / box
    geom = lpc.geometry(0, nm, box)
    ws = lpc.workspace(geom, lpc.LPC_OP_BISPECTRUM, n_particles=n)
    pos_d = to_dev(pos)
    tri = [t for t in TRIANGLES if max(t) + dk / 2 < np.pi * nm / box]  # shells below the mesh's Nyquist
    B, Q, P = lpc.lpc_bispectrum(geom, pos_d, tri, dk, ws)
    B2, Q2, P2 = lpc.lpc_bispectrum(geom, pos_d, tri, dk, ws)
    assert np.array_equal(B, B2) and np.array_equal(Q, Q2) and np.array_equal(P, P2)  # fixed reduction order
    dhat = obs.delta_hat_from_particles(pos, nm, box)
    worst = 0.0
    for t, b, q, p in zip(tri, B, Q, P):
        rb, rq = obs.bispectrum(dhat, box, *t, dk)
        rp = [obs.power_in_shell(dhat, box, kc, dk) for kc in t]
        err = max(abs(b / rb - 1), abs(q / rq - 1), *(abs(x / y - 1) for x, y in zip(p, rp)))
        worst = max(worst, err)
        assert err < REL, (t, b, rb, q, rq)
    say(f"bispectrum nm={nm}: {len(tri)} triangles, worst relative error {worst:.2e}")


def test_unclosed_shells_give_nan_and_arguments_are_checked():
    from paper_1506_03737_amd import lpc
    nm, box, n = 32, 300.0, 5000
    pos_d = to_dev(synth.clustered_positions(3, n, box))
    geom = lpc.geometry(0, nm, box)
    ws = lpc.workspace(geom, lpc.LPC_OP_BISPECTRUM, n_particles=n)
    dk = 2 * np.pi / box
    B, Q, _ = lpc.lpc_bispectrum(geom, pos_d, [(0.05, 0.05, 0.3)], dk, ws)  # k3 > k1 + k2 + dk: no triangle closes
    assert np.isnan(B[0]) and np.isnan(Q[0])
    for tri, d in (([(0.1, 0.1, 0.0)], dk), ([(0.1, 0.1, 0.1)], 0.0), ([(0.1, 0.1, 0.1)] * 257, dk)):
        with pytest.raises(lpc.LpcError):
            lpc.lpc_bispectrum(geom, pos_d, tri, d, ws)
