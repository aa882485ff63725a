"""Pins for oracle/cosmology.py: Einstein-de Sitter closed forms, the growth ODEs, resume additivity.

Each check is chosen so that a plausible mistake (a dropped factor of a^2 E in a kick, a wrong power in the drift, a
wrong derivative of Eq. 7, a mis-normalised D1) fails it.
"""
import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle import cosmology as C

A_LIST = [0.1 + 0.09 * i for i in range(11)]


@pytest.mark.parametrize("a", [0.05, 0.1, 0.37, 0.82, 1.0])
def test_eds_growth_closed_forms(a):
    # Omega_m = 1: D1 = a, D2 = -(3/7) a^2, D1' = 1, D2' = -(6/7) a, E = a^(-3/2).
    assert C.growth_D1(a, 1.0) == pytest.approx(a, rel=1e-12)
    assert C.growth_D2(a, 1.0) == pytest.approx(-3.0 / 7.0 * a * a, rel=1e-12)
    assert C.growth_dD1_da(a, 1.0) == pytest.approx(1.0, rel=1e-12)
    assert C.growth_dD2_da(a, 1.0) == pytest.approx(-6.0 / 7.0 * a, rel=1e-12)
    f1, f2 = C.frame_momentum_factors(a, 1.0)
    assert f1 == pytest.approx(a**1.5, rel=1e-12)
    assert f2 == pytest.approx(-6.0 / 7.0 * a**2.5, rel=1e-12)


@pytest.mark.parametrize("i", [0, 3, 10])
def test_eds_kick_drift_closed_forms(i):
    lo, hi = C.half_points(A_LIST)
    a = A_LIST[i]
    # standard: K = int a^-2 a^(3/2) = 2 (sqrt(a+) - sqrt(a-)); Q = int a^(-3/2) = 2 (a_i^-1/2 - a_{i+1}^-1/2)
    assert C.kick_factor(lo[i], a, hi[i], 1.0, False, -2.5) == pytest.approx(2 * (hi[i] ** 0.5 - lo[i] ** 0.5),
                                                                            rel=1e-12, abs=1e-15)
    n = -2.5
    assert C.kick_factor(lo[i], a, hi[i], 1.0, True, n) == pytest.approx(
        (hi[i] ** n - lo[i] ** n) / (n * a ** (n - 0.5)), rel=1e-12, abs=1e-15)
    if i < 10:
        b = A_LIST[i + 1]
        assert C.drift_factor(a, b, 1.0, False, n) == pytest.approx(2 * (a**-0.5 - b**-0.5), rel=1e-12)
        mid = 0.5 * (a + b)
        assert C.drift_factor(a, b, 1.0, True, n) == pytest.approx(
            (b ** (n - 0.5) - a ** (n - 0.5)) / ((n - 0.5) * mid**n), rel=1e-12)


def _growth_odes(om):
    def rhs(a, y):
        E = C.hubble_E(a, om)
        dlnE = C.dE_da(a, om) / E
        src = 1.5 * om / (a**5 * E**2)
        d1, v1, d2, v2 = y
        return [v1, -(3.0 / a + dlnE) * v1 + src * d1, v2, -(3.0 / a + dlnE) * v2 + src * (d2 - d1 * d1)]
    return rhs


@pytest.mark.parametrize("om", [0.31, 0.25])
def test_lcdm_growth_against_ode(om):
    """D1 from the Heath integral == the growing solution of the linear growth ODE; D2 (Eq. 7) close to the 2LPT ODE."""
    a0 = 1e-4
    sol = solve_ivp(_growth_odes(om), (a0, 1.0), [a0, 1.0, -3 / 7 * a0**2, -6 / 7 * a0],
                    rtol=1e-12, atol=1e-20, dense_output=True, method="DOP853")
    norm = sol.sol(1.0)[0]
    for a in [0.1, 0.3, 0.55, 1.0]:
        d1, v1, d2, _ = sol.sol(a)
        assert C.growth_D1(a, om) == pytest.approx(d1 / norm, rel=1e-9)
        assert C.growth_dD1_da(a, om) == pytest.approx(v1 / norm, rel=1e-9)
        # Bouchet's fit against the exact second-order growth: agreement well below a percent.
        assert C.growth_D2(a, om) == pytest.approx(d2 / norm**2, rel=3e-3)


@pytest.mark.parametrize("a", [0.15, 0.5, 0.9])
def test_growth_identities_and_derivatives(a):
    om = 0.31
    h = 1e-5
    # D2' is the derivative of Eq. 7
    fd = (C.growth_D2(a + h, om) - C.growth_D2(a - h, om)) / (2 * h)
    assert C.growth_dD2_da(a, om) == pytest.approx(fd, rel=1e-8)
    # d/da (a^3 E D1') = (3/2) Om D1 / (a^2 E)
    g = lambda x: x**3 * C.hubble_E(x, om) * C.growth_dD1_da(x, om)
    lhs = (g(a + h) - g(a - h)) / (2 * h)
    rhs = 1.5 * om * C.growth_D1(a, om) / (a**2 * C.hubble_E(a, om))
    assert lhs == pytest.approx(rhs, rel=1e-7)


@pytest.mark.parametrize("modified", [False, True])
def test_half_kicks_add_up(modified):
    """Resume additivity: closing half kick at a_k plus opening half kick at a_k == the full kick at a_k."""
    om = 0.31
    lo, hi = C.half_points(A_LIST)
    for k in (1, 5, 9):
        full = C.kick_factor(lo[k], A_LIST[k], hi[k], om, modified, -2.5)
        close = C.kick_factor(lo[k], A_LIST[k], A_LIST[k], om, modified, -2.5)
        open_ = C.kick_factor(A_LIST[k], A_LIST[k], hi[k], om, modified, -2.5)
        assert close + open_ == pytest.approx(full, rel=1e-13)


def test_coefficient_table_shape_and_last_row():
    tab = C.coefficient_table(A_LIST, 0.31)
    col = {n: i for i, n in enumerate(C.COEF_COLUMNS)}
    assert tab.shape == (11, len(C.COEF_COLUMNS))
    assert tab[-1, col["Q"]] == 0.0 and tab[-1, col["dDD1"]] == 0.0
    assert np.all(tab[:-1, col["Q"]] > 0) and np.all(tab[:, col["K"]] > 0)
    # D1 increases, D2 decreases (D2 < 0)
    assert np.all(np.diff(tab[:, col["D1"]]) > 0) and np.all(np.diff(tab[:, col["D2"]]) < 0)
