"""GPU parity of the hand-written 3-D r2c/c2r FFT against brute force and the oracle's FP64 transforms.

Tolerance: FP32 arithmetic with O(log n) error growth; relative L2 error <= 2e-6 * log2(n) and the max error below
1e-5 of the largest coefficient (derived from float32 epsilon 6e-8 times the stage count with margin).
"""
import numpy as np
import pytest

import synth
from oracle import dft
from tests.gpu_util import HAVE_GPU, rel_l2, requires_gpu, say, to_dev, to_np, torch

pytestmark = [pytest.mark.gpu, requires_gpu]


def gpu_r2c(lpc, f):
    n = f.shape[0]
    pitch = lpc.lpc_fft_pitch(n)
    out = torch.empty((n, n, pitch, 2), dtype=torch.float32, device="cuda")
    ws = lpc.workspace(lpc.geometry(n, n, 1.0), lpc.LPC_OP_FFT)
    lpc.lpc_fft_r2c(n, to_dev(f.astype(np.float32)), out, ws)
    o = to_np(out)
    return o.view(np.complex64)[..., 0][:, :, : n // 2 + 1]


def gpu_c2r(lpc, F):
    n = F.shape[0]
    pitch = lpc.lpc_fft_pitch(n)
    buf = np.zeros((n, n, pitch, 2), dtype=np.float32)
    buf[:, :, : n // 2 + 1, 0] = F.real
    buf[:, :, : n // 2 + 1, 1] = F.imag
    out = torch.empty((n, n, n), dtype=torch.float32, device="cuda")
    ws = lpc.workspace(lpc.geometry(n, n, 1.0), lpc.LPC_OP_FFT)
    lpc.lpc_fft_c2r(n, to_dev(buf), out, ws)
    return to_np(out)


def test_r2c_matches_brute_force_8():
    from paper_1506_03737_amd import lpc
    say("fft: r2c n=8 vs brute-force DFT")
    f = synth.random_real_mesh(1, (8, 8, 8))
    ref = dft.dft3_brute(f.astype(np.float64))[:, :, :5]
    got = gpu_r2c(lpc, f)
    assert rel_l2(got, ref) < 1e-6


@pytest.mark.parametrize("n", [8, 10, 12, 16, 20, 24, 30, 32, 40, 48, 60, 64, 96, 128, 160, 192, 250, 256, 320, 384])
def test_r2c_and_c2r_match_numpy(n):
    from paper_1506_03737_amd import lpc
    say(f"fft: r2c/c2r n={n}")
    f = synth.random_real_mesh(n, (n, n, n))
    ref = np.fft.rfftn(f.astype(np.float64))
    got = gpu_r2c(lpc, f)
    tol = 2e-6 * np.log2(n)
    assert rel_l2(got, ref) < tol
    assert np.abs(got - ref).max() < 1e-5 * np.abs(ref).max() * np.log2(n)
    back = gpu_c2r(lpc, ref.astype(np.complex64))
    assert rel_l2(back, np.fft.irfftn(ref, s=(n,) * 3, axes=(0, 1, 2)) * n**3) < tol


def test_c2r_of_single_mode():
    """A single Hermitian pair (k = (1, 2, 3)) inverts to 2 cos(2 pi k.x / n) exactly (up to FP32)."""
    from paper_1506_03737_amd import lpc
    n = 24
    say("fft: c2r single mode n=24")
    F = np.zeros((n, n, n // 2 + 1), dtype=np.complex64)
    F[1, 2, 3] = 1.0
    x = np.arange(n)
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    ref = 2 * np.cos(2 * np.pi * (X + 2 * Y + 3 * Z) / n)
    assert np.abs(gpu_c2r(lpc, F) - ref).max() < 1e-5


@pytest.mark.parametrize("n", [768, 1024])
def test_full_size_round_trip_and_sampled_modes(n):
    """Full mesh sizes of the single-box workloads: c2r(r2c(f)) = n^3 f, and sampled modes equal direct sums."""
    from paper_1506_03737_amd import lpc
    say(f"fft: full-size round trip n={n}")
    rng = np.random.default_rng(n)
    f = rng.standard_normal((n, n, n), dtype=np.float32)
    F = gpu_r2c(lpc, f)
    flat = f.reshape(n * n, n)
    for kx, ky, kz in [(0, 0, 1), (3, n - 5, 17), (n // 2, 7, n // 2), (n - 1, n // 3, 100)]:
        ph = lambda k: np.exp(-2j * np.pi * k * np.arange(n) / n)
        ez = ph(kz)
        # sum over z in float32 (1e3 terms), the rest in float64
        sz = (flat @ ez.real.astype(np.float32)).astype(np.float64) + 1j * (flat @ ez.imag.astype(np.float32))
        direct = ph(kx) @ (sz.reshape(n, n) @ ph(ky))
        assert abs(F[kx, ky, kz] - direct) < 2e-5 * np.sqrt(f.size)
    back = gpu_c2r(lpc, F)
    back /= float(n) ** 3
    assert np.abs(back - f).max() < 1e-4
