"""Pins of the Gilbarg-Paolucci shock-structure oracle (oracle/shock.py) against
what the paper and the mathematics fix: the end states are the Rankine-Hugoniot
states; the thickness (eq. ShockThickness) reproduces the paper's printed table
at Pr = 1 (the paper's setting) and not at Pr = 2/3 (the coefficient its printed
equations carry); the traced profile satisfies both ODEs."""
import os

import numpy as np
import pytest

from oracle.shock import GPShock

HERE = os.path.dirname(os.path.abspath(__file__))
GAMMA = 5.0 / 3.0


def _rh(M, g=GAMMA):
    rho = (g + 1) * M * M / ((g - 1) * M * M + 2)
    T = (2 * g * M * M - (g - 1)) * ((g - 1) * M * M + 2) / ((g + 1) ** 2 * M * M)
    return rho, T


@pytest.mark.parametrize("M", [1.2, 2.0, 3.0, 4.0, 6.0])
def test_end_states_are_rankine_hugoniot(M):
    s = GPShock(M)
    rho1, T1 = _rh(M)
    assert np.isclose(s.Om_inf / s.Om_1, rho1, rtol=1e-12)
    assert np.isclose(s.th_1 / s.th_inf, T1, rtol=1e-12)
    # both are zeros of both right-hand sides
    for Om, th in ((s.Om_inf, s.th_inf), (s.Om_1, s.th_1)):
        assert abs(s.dOm_dz(Om, th)) < 1e-12 and abs(s.dth_dz(Om, th)) < 1e-12
    # the separatrix traced from the downstream saddle arrives at the upstream state
    assert abs(s.theta_of_omega(s.Om_hi) - s.th_inf) < 1e-6 * s.th_inf


def _table():
    rows = [ln.split() for ln in open(os.path.join(HERE, "golden", "shock_thickness_table.txt"))
            if ln.strip() and not ln.startswith("#")]
    return [tuple(float(v) for v in r) for r in rows]


def _mean_free_path_mm():
    T, p, R, mu, delta = 300.0, 41.4, 208.0, 2.688e-5, 5.0
    rho = p / (R * T)
    return 1e3 * (16.0 / delta) * mu / (rho * np.sqrt(2 * np.pi * R * T))


def test_thickness_reproduces_the_paper_table():
    lam = _mean_free_path_mm()
    assert abs(lam - 0.207) < 5e-4
    for M, D_mm, Re, Kn in _table():
        s = GPShock(M, Pr=1.0, s_visc=0.5, delta=5.0)
        D = D_mm / lam
        # three printed digits: 0.5 in the last place
        assert abs(s.thickness - D) <= 0.5e-3 / lam * 1.01 + 1e-12, (M, s.thickness, D)
        # Re_Delta = rho u Delta / mu = (Delta / l_inf) / mu_h_inf; Kn_Delta = l_inf / Delta
        assert abs(s.thickness / s.mu_inf - Re) <= 0.006 * Re, (M, s.thickness / s.mu_inf, Re)
        assert abs(1.0 / s.thickness - Kn) <= 0.0006 + 1e-3 * Kn, (M, 1 / s.thickness, Kn)


def test_thickness_discriminates_the_prandtl_number():
    lam = _mean_free_path_mm()
    M, D_mm, _, _ = _table()[1]
    s = GPShock(M, Pr=2.0 / 3.0)
    assert abs(s.thickness / (D_mm / lam) - 1) > 0.1


@pytest.mark.parametrize("M", [1.2, 4.0])
def test_profile_satisfies_both_odes(M):
    s = GPShock(M)
    z = np.linspace(-2.0, 2.0, 9) * s.thickness
    h = 1e-4 * s.thickness
    rho_p, u_p, T_p = s.profile(z + h)
    rho_m, u_m, T_m = s.profile(z - h)
    rho, u, T = s.profile(z)
    Om, th = u * s.Om_inf, T * s.th_inf
    dOm = (u_p - u_m) * s.Om_inf / (2 * h)
    dth = (T_p - T_m) * s.th_inf / (2 * h)
    scale_O = s.max_slope
    assert np.all(np.abs(dOm - s.dOm_dz(Om, th)) <= 1e-5 * scale_O)
    assert np.all(np.abs(dth - s.dth_dz(Om, th)) <= 1e-5 * scale_O)
    # mass flux and monotone velocity; the steepest point at z = 0
    assert np.allclose(rho * u, 1.0, rtol=1e-13)
    assert np.all(np.diff(u) < 0)
    _, u0, _ = s.profile(np.array([0.0]))
    assert np.isclose(u0[0] * s.Om_inf, s.Om_star, rtol=1e-8)
