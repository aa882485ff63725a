"""Shared helpers of the GPU parity tests (device arrays in, NumPy out). Holds none of the method's arithmetic."""
import sys

import numpy as np
import pytest

try:
    import torch
    HAVE_GPU = torch.cuda.is_available()
except Exception:  # pragma: no cover
    torch = None
    HAVE_GPU = False

requires_gpu = pytest.mark.skipif(not HAVE_GPU, reason="needs a GPU")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def dev():
    return torch.device("cuda:0")


def to_dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(dev())


def to_np(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def particle_set(lpc, pos, vel, psi1, psi2):
    n = pos.shape[1]
    return lpc.ParticleSet(to_dev(pos.astype(np.float32)), to_dev(vel.astype(np.float32)),
                           to_dev(psi1.astype(np.float32)), to_dev(psi2.astype(np.float32)),
                           torch.arange(n, dtype=torch.int32, device=dev()))


def periodic_diff(a, b, box):
    d = np.asarray(a, dtype=np.float64) - np.asarray(b, dtype=np.float64)
    return d - box * np.round(d / box)


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.complex128 if np.iscomplexobj(a) else np.float64)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(np.asarray(b).ravel()), 1e-300))
