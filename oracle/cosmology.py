"""Background cosmology, growth factors and the KDK time-step factors, in float64.

Oracle (test infrastructure only). Follows Sec. 2.1 (Eq. 7: Bouchet second-order growth), Sec. 2.3 (Eq. 16: the
Quinn et al. kick/drift factors; Eq. 19: the modified COLA factors with nLPT) of Howlett, Manera & Percival (2015).

Units: lengths in Mpc/h, time variable is the scale factor a, H0 = 1. The universe is flat: Omega_L = 1 - Omega_m.

Readings taken where the paper is silent or garbled:
  * D1 is the growing mode normalised to D1(1) = 1 (the stored displacements are the z = 0 ones, Sec. 2.2). It is
    computed from the Heath integral D1 ~ E(a) int_0^a da'/(a' E(a'))^3, which the paper does not print.
  * D2 is the Bouchet approximation of Eq. 7 (the only D2 formula the paper writes; the Matsubara form it also names
    is not given).
  * The momentum is p = a^2 dx/dt / H0 (Mpc/h). Then dp/da = -(3/2) Om grad(psi) / (a^2 E) with lap(psi) = delta,
    and dx/da = p / (a^3 E). The kick factor therefore carries 1/(a^2 E) and the drift factor 1/(a^3 E); the paper's
    Eq. 16 prefactor H0/a_i and the missing 1/(a_i^2 E(a_i)) of Eq. 19's kick are read this way.
  * nLPT defaults to -2.5 (the value stated in Sec. 1 and Sec. 7.3; Eq. 19's text says +2.5).
  * The LPT frame acceleration uses the growth-equation identities
        d/da (a^3 E D1') = (3/2) Om D1 / (a^2 E),   d/da (a^3 E D2') = (3/2) Om (D2 - D1^2) / (a^2 E),
    with D1, D2 evaluated as above.
"""
import numpy as np
from scipy import integrate


def hubble_E(a, omega_m):
    """E(a) = H(a)/H0 = sqrt(Om a^-3 + 1 - Om) for a flat universe."""
    a = np.asarray(a, dtype=np.float64)
    return np.sqrt(omega_m / a**3 + (1.0 - omega_m))


def dE_da(a, omega_m):
    """dE/da = -3 Om / (2 a^4 E)."""
    return -1.5 * omega_m / (a**4 * hubble_E(a, omega_m))


def _heath_integral(a, omega_m):
    """int_0^a da' / (a' E(a'))^3, by adaptive quadrature (QUADPACK)."""
    f = lambda x: 1.0 / (x * hubble_E(x, omega_m)) ** 3
    val, _ = integrate.quad(f, 0.0, float(a), epsabs=0.0, epsrel=2e-14, limit=200)
    return val


def growth_D1(a, omega_m):
    """Linear growth factor D1(a), normalised to D1(1) = 1 (Sec. 2.1, Eq. 5; normalisation read from Sec. 2.2)."""
    norm = hubble_E(1.0, omega_m) * _heath_integral(1.0, omega_m)
    return float(hubble_E(a, omega_m) * _heath_integral(a, omega_m) / norm)


def growth_dD1_da(a, omega_m):
    """dD1/da = (E'/E) D1 + 1 / (a^3 E^2 norm), differentiating the Heath integral form."""
    norm = hubble_E(1.0, omega_m) * _heath_integral(1.0, omega_m)
    E = hubble_E(a, omega_m)
    d1 = E * _heath_integral(a, omega_m) / norm
    return float(dE_da(a, omega_m) / E * d1 + 1.0 / (a**3 * E**2 * norm))


def omega_m_of_a(a, omega_m):
    """Om(a) = Om / (Om + OL a^3)."""
    return omega_m / (omega_m + (1.0 - omega_m) * a**3)


def growth_D2(a, omega_m):
    """Second-order growth factor, Bouchet et al. approximation (Sec. 2.1, Eq. 7): D2 = -(3/7) D1^2 Om(a)^(-1/143)."""
    d1 = growth_D1(a, omega_m)
    return float(-3.0 / 7.0 * d1**2 * omega_m_of_a(a, omega_m) ** (-1.0 / 143.0))


def growth_dD2_da(a, omega_m):
    """Analytic derivative of Eq. 7, using dOm(a)/da = -3 Om(a) (1 - Om(a)) / a."""
    d1 = growth_D1(a, omega_m)
    dd1 = growth_dD1_da(a, omega_m)
    om_a = omega_m_of_a(a, omega_m)
    dom = -3.0 * om_a * (1.0 - om_a) / a
    g = om_a ** (-1.0 / 143.0)
    dg = (-1.0 / 143.0) * om_a ** (-1.0 / 143.0 - 1.0) * dom
    return float(-3.0 / 7.0 * (2.0 * d1 * dd1 * g + d1**2 * dg))


def _quad(f, lo, hi):
    val, _ = integrate.quad(f, float(lo), float(hi), epsabs=0.0, epsrel=2e-14, limit=200)
    return val


def kick_factor(a_lo, a_i, a_hi, omega_m, modified, n_lpt):
    """Kick factor K such that p_{i+1/2} = p_{i-1/2} + K * F(a_i), where dp/da = F / (a^2 E) (Sec. 2.3).

    Standard (Eq. 16): K = int_{a_lo}^{a_hi} da / (a^2 E).
    Modified (Eq. 19): the residual momentum is taken to grow like u(a) = a^nLPT over the kick, so
        K = [u(a_hi) - u(a_lo)] / (u'(a_i) a_i^2 E(a_i)).
    """
    if modified:
        u = lambda a: a**n_lpt
        du = n_lpt * a_i ** (n_lpt - 1.0)
        return (u(a_hi) - u(a_lo)) / (du * a_i**2 * float(hubble_E(a_i, omega_m)))
    return _quad(lambda a: 1.0 / (a**2 * hubble_E(a, omega_m)), a_lo, a_hi)


def drift_factor(a_i, a_ip1, omega_m, modified, n_lpt):
    """Drift factor Q such that x_{i+1} = x_i + Q * p_{i+1/2} (+ the LPT displacement change) (Sec. 2.3).

    Standard (Eq. 16): Q = int_{a_i}^{a_{i+1}} da / (a^3 E).
    Modified (Eq. 19): Q = int_{a_i}^{a_{i+1}} u(a) / (a^3 E) da / u(a_{i+1/2}), u = a^nLPT, a_{i+1/2} the midpoint.
    """
    if modified:
        a_mid = 0.5 * (a_i + a_ip1)
        val = _quad(lambda a: a**n_lpt / (a**3 * hubble_E(a, omega_m)), a_i, a_ip1)
        return val / a_mid**n_lpt
    return _quad(lambda a: 1.0 / (a**3 * hubble_E(a, omega_m)), a_i, a_ip1)


def frame_momentum_factors(a, omega_m):
    """Factors (f1, f2) with p_LPT = f1 Psi1 + f2 Psi2 = a^3 E (D1' Psi1 + D2' Psi2) (Sec. 2.3, frame velocity)."""
    pref = a**3 * float(hubble_E(a, omega_m))
    return pref * growth_dD1_da(a, omega_m), pref * growth_dD2_da(a, omega_m)


def half_points(a_list):
    """Kick interval ends: a_{i-1/2}, a_{i+1/2} as arithmetic midpoints, with a_{-1/2} = a_0 and a_{N+1/2} = a_N."""
    a = np.asarray(a_list, dtype=np.float64)
    lo = np.empty_like(a)
    hi = np.empty_like(a)
    lo[0] = a[0]
    lo[1:] = 0.5 * (a[:-1] + a[1:])
    hi[-1] = a[-1]
    hi[:-1] = 0.5 * (a[:-1] + a[1:])
    return lo, hi


# Column order of the per-time coefficient table (one row per a_i in the time list).
COEF_COLUMNS = ("a", "D1", "D2", "dD1", "dD2", "E", "K", "Q", "dDD1", "dDD2", "f1", "f2")


def coefficient_table(a_list, omega_m, modified=True, n_lpt=-2.5):
    """Per-time FP64 table used by one COLA run over a_list (rows i = 0..N).

    K[i]  : kick factor for the kick at a_i, from a_{i-1/2} to a_{i+1/2}.
    Q[i]  : drift factor from a_i to a_{i+1} (0 in the last row: no drift after the closing half kick).
    dDD1/dDD2[i] : D(a_{i+1}) - D(a_i) (0 in the last row).
    f1/f2[i] : frame momentum factors a^3 E D'(a_i).
    """
    a = np.asarray(a_list, dtype=np.float64)
    n = a.size
    lo, hi = half_points(a)
    tab = np.zeros((n, len(COEF_COLUMNS)), dtype=np.float64)
    for i in range(n):
        ai = a[i]
        d1, d2 = growth_D1(ai, omega_m), growth_D2(ai, omega_m)
        f1, f2 = frame_momentum_factors(ai, omega_m)
        K = kick_factor(lo[i], ai, hi[i], omega_m, modified, n_lpt)
        if i + 1 < n:
            Q = drift_factor(ai, a[i + 1], omega_m, modified, n_lpt)
            dd1 = growth_D1(a[i + 1], omega_m) - d1
            dd2 = growth_D2(a[i + 1], omega_m) - d2
        else:
            Q = dd1 = dd2 = 0.0
        tab[i] = (ai, d1, d2, growth_dD1_da(ai, omega_m), growth_dD2_da(ai, omega_m), float(hubble_E(ai, omega_m)),
                  K, Q, dd1, dd2, f1, f2)
    return tab
