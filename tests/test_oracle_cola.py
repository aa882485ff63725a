"""Pins for oracle/cola.py: the 1-D plane-wave Zel'dovich solution (exact before shell crossing).

For Psi1 = A sin(2 pi q_x / L) x_hat and Psi2 = 0, the Zel'dovich trajectory x = q + D1(a) Psi1 is an exact solution
of the equation of motion in 1-D, and the exact gravitational field there is grad(psi) = q - x (the mass to the left
of a particle is conserved). So:
  * with that exact force, plain KDK (cola = 0) converges to the trajectory at second order in the step;
  * with that exact force, COLA keeps the trajectory to rounding (the residual force vanishes identically);
  * with the PM force on a mesh, COLA stays within a small fraction of a cell of it.
"""
import numpy as np
import pytest

from oracle import cola, cosmology, ic

OM = 0.31
L = 256.0


def plane_wave(n_side, amp_frac=0.5):
    q = ic.lattice_positions(n_side, L)
    amp = amp_frac * L / (2 * np.pi)          # D1(1) * A * 2 pi / L = amp_frac < 1: no shell crossing by a = 1
    psi1 = np.zeros_like(q)
    psi1[0] = amp * np.sin(2 * np.pi * q[0] / L)
    return q, psi1, np.zeros_like(q)


def exact_force(q):
    def f(x, a):
        d = q - x
        return d - L * np.round(d / L)
    return f


def za_state(q, psi1, a):
    d1 = cosmology.growth_D1(a, OM)
    f1, _ = cosmology.frame_momentum_factors(a, OM)
    return q + d1 * psi1, f1 * psi1


def run(q, psi1, psi2, n_steps, cola_on, modified, force_fn=None, n_mesh=64):
    a_list = np.linspace(0.1, 1.0, n_steps + 1)
    x0, p0 = za_state(q, psi1, a_list[0])
    return cola.cola_run(x0, p0, psi1, psi2, a_list, OM, n_mesh, L, cola=cola_on, modified=modified,
                         force_fn=force_fn)


@pytest.mark.parametrize("modified", [False, True])
def test_plain_kdk_converges_second_order(modified):
    q, psi1, psi2 = plane_wave(8)
    xt, pt = za_state(q, psi1, 1.0)
    errs = []
    for n in (10, 20, 40):
        x, p = run(q, psi1, psi2, n, False, modified, exact_force(q))
        errs.append(np.abs(x - xt).max())
    assert errs[0] > 1e-6                       # the plain integrator is not exact ...
    for e0, e1 in zip(errs[:-1], errs[1:]):     # ... but second order
        assert 3.3 < e0 / e1 < 4.7


@pytest.mark.parametrize("modified", [False, True])
def test_cola_exact_force_keeps_zeldovich(modified):
    q, psi1, psi2 = plane_wave(8)
    x, p = run(q, psi1, psi2, 10, True, modified, exact_force(q))
    xt, pt = za_state(q, psi1, 1.0)
    assert np.abs(x - xt).max() < 1e-10 * L
    assert np.abs(p - pt).max() < 1e-10 * np.abs(pt).max()


def _pm_plane_wave_error(n_side, n_mesh):
    q, psi1, psi2 = plane_wave(n_side)
    x, p = run(q, psi1, psi2, 10, True, True, n_mesh=n_mesh)
    xt, _ = za_state(q, psi1, 1.0)
    d = x - xt
    d -= L * np.round(d / L)
    return np.abs(d).max()


def test_cola_pm_force_plane_wave_converges_under_refinement():
    """PM force with Nm = N: the error against the exact trajectory is a small fraction of a cell (the displacement
    itself is 20 Mpc/h = 2.5 cells at N = 32) and falls as the mesh and particle lattice are refined together."""
    e16, e32, e64 = (_pm_plane_wave_error(n, n) for n in (16, 32, 64))
    assert e32 < 0.15 * (L / 32)
    assert e16 / e32 > 1.6 and e32 / e64 > 1.6


def test_cola_pm_force_plane_wave_fine_mesh():
    """Nm = 3N (the particles start at cell centres): below 0.75 of a fine cell, against a displacement of 7.5 fine
    cells; a mesh finer than the particle lattice feels sheet discreteness, so this bound is looser than at Nm = N."""
    assert _pm_plane_wave_error(32, 96) < 0.75 * (L / 96)


def test_split_run_equals_single_run():
    """Resume: one run over a[0..10] == runs over a[0..5] then a[5..10] (the half kicks at a_5 add up)."""
    q, psi1, _ = plane_wave(8)
    rng = np.random.default_rng(0)
    psi2 = 0.3 * rng.standard_normal(q.shape)
    psi1 = psi1 + rng.standard_normal(q.shape)
    a = np.linspace(0.1, 1.0, 11)
    x0, p0 = za_state(q, psi1, a[0])
    kw = dict(omega_m=OM, n_mesh=16, box=L)
    x1, p1 = cola.cola_run(x0, p0, psi1, psi2, a, **kw)
    xa, pa = cola.cola_run(x0, p0, psi1, psi2, a[:6], **kw)
    xb, pb = cola.cola_run(xa, pa, psi1, psi2, a[5:], **kw)
    assert np.allclose(x1, xb, atol=1e-9) and np.allclose(p1, pb, atol=1e-9)
