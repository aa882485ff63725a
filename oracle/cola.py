"""The COLA kick-drift-kick integrator about the stored 2LPT displacements, in float64.

Oracle (test infrastructure only). Follows Sec. 2.2 (Eq. 11: the equation of motion split into the residual and the
2LPT frame) and Sec. 2.3 (Eqs. 14-19: kick-drift-kick, the COLA kick and drift, zero initial residual momentum with
the frame momentum removed at the start and added back at the end) of Howlett, Manera & Percival (2015).

Schedule for a time list a_0 < a_1 < ... < a_N (readings: midpoints a_{i+1/2} = (a_i + a_{i+1}) / 2, opening and
closing half kicks, N drifts and N + 1 force evaluations):
    remove frame momentum at a_0            p_res = p - (f1(a_0) Psi1 + f2(a_0) Psi2)
    for i = 0 .. N:
        force at a_i                        g = grad(psi)(x)
        kick a_{i-1/2} -> a_{i+1/2}         p_res += K_i * (-(3/2) Om) [g + D1(a_i) Psi1 + (D2(a_i) - D1(a_i)^2) Psi2]
        drift a_i -> a_{i+1} (i < N)        x += Q_i p_res + dD1_i Psi1 + dD2_i Psi2, wrapped into [0, L)
    add frame momentum at a_N               p = p_res + f1(a_N) Psi1 + f2(a_N) Psi2
With cola = 0 this is the plain PM integrator: no frame terms, the kick uses g alone and the drift Q p alone.
"""
import numpy as np

from . import cosmology as cosmo
from .pm import pm_force


def kick_acceleration(g, psi1, psi2, omega_m, d1, d2, cola):
    """The force term F of dp_res/da = F / (a^2 E): -(3/2) Om [g + D1 Psi1 + (D2 - D1^2) Psi2] (Sec. 2.3)."""
    if cola:
        return -1.5 * omega_m * (g + d1 * psi1 + (d2 - d1 * d1) * psi2)
    return -1.5 * omega_m * g


def cola_run(pos, vel, psi1, psi2, a_list, omega_m, n_mesh, box, cola=True, modified=True, n_lpt=-2.5,
             deconv_power=1, force_fn=None):
    """Advance particles over a_list. Arrays are (3, n) float64; returns (pos, vel) at a_list[-1].

    force_fn(pos, a) -> (3, n) may replace the PM force (used by the integrator pins); default is pm.pm_force.
    """
    if force_fn is None:
        force_fn = lambda x, a: pm_force(x, n_mesh, box, deconv_power)
    x = np.array(pos, dtype=np.float64)
    p = np.array(vel, dtype=np.float64)
    psi1 = np.asarray(psi1, dtype=np.float64)
    psi2 = np.asarray(psi2, dtype=np.float64)
    tab = cosmo.coefficient_table(a_list, omega_m, modified, n_lpt)
    col = {name: k for k, name in enumerate(cosmo.COEF_COLUMNS)}
    if cola:
        p = p - (tab[0, col["f1"]] * psi1 + tab[0, col["f2"]] * psi2)
    n_last = tab.shape[0] - 1
    for i in range(n_last + 1):
        row = tab[i]
        g = force_fn(x, row[col["a"]])
        acc = kick_acceleration(g, psi1, psi2, omega_m, row[col["D1"]], row[col["D2"]], cola)
        p = p + row[col["K"]] * acc
        if i < n_last:
            x = x + row[col["Q"]] * p
            if cola:
                x = x + row[col["dDD1"]] * psi1 + row[col["dDD2"]] * psi2
            x = np.mod(x, box)
    if cola:
        p = p + tab[n_last, col["f1"]] * psi1 + tab[n_last, col["f2"]] * psi2
    return x, p
