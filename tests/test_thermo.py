"""Set-up helpers of the convection cell (paper_1111_0905_amd/thermo.py),
checked against their defining equations: the Rayleigh number with the
adiabatic correction (Table 1 caption), the liquid spinodal, the hydrostatic
liquid column, and against the oracle's independent EOS where both exist."""
import math

import pytest

from oracle import eos
from paper_1111_0905_amd import thermo

TC = 0.08
G = thermo.coupling_for_tc(TC)


def _ra(g, L, rho, T_d, T_u, tau_nu, tau_kappa, rho_kappa=0.5, c_v=1.0):
    T = 0.5 * (T_d + T_u)
    b, c = thermo.beta(rho, T, G), thermo.cp(rho, T, G, c_v)
    chi = thermo.kappa(tau_kappa, rho_kappa, c_v) / (rho * c)
    nu = (tau_nu - 0.5) / 3.0
    return g * b * L ** 4 * ((T_d - T_u) / L - b * T * g / c) / (chi * nu)


def test_eos_agrees_with_oracle():
    for rho in (0.5, 1.0, 1.9, 2.49):
        for t in (0.85, 0.9, 0.95):
            T = t * TC
            assert math.isclose(thermo.pressure(rho, T, G), eos.pressure(rho, T, G), rel_tol=1e-14)
    assert math.isclose(-G / math.e ** 2, TC, rel_tol=1e-15)


@pytest.mark.parametrize("Ra", [1e5, 5e5])
def test_gravity_for_rayleigh_inverts_the_definition(Ra):
    L, rho, T_d, T_u = 128, 1.75, 0.95 * TC, 0.85 * TC
    g = thermo.gravity_for_rayleigh(Ra, L, rho, T_d, T_u, G, 0.5495, 0.65)
    assert math.isclose(_ra(g, L, rho, T_d, T_u, 0.5495, 0.65), Ra, rel_tol=1e-9)
    # the smaller root: below the g of maximum Ra
    ramax = thermo.max_rayleigh(L, rho, T_d, T_u, G, 0.5495, 0.65)
    assert _ra(1.01 * g, L, rho, T_d, T_u, 0.5495, 0.65) > Ra
    assert Ra < ramax
    with pytest.raises(ValueError):
        thermo.gravity_for_rayleigh(1.01 * ramax, L, rho, T_d, T_u, G, 0.5495, 0.65)


def test_prandtl_and_spinodal():
    nu, rho, T = 0.0165, 2.0, 0.9 * TC
    tk = thermo.tau_kappa_for_prandtl(9.0, nu, rho, T, G)
    chi = thermo.kappa(tk, 0.5) / (rho * thermo.cp(rho, T, G))
    assert math.isclose(nu / chi, 9.0, rel_tol=1e-12)
    rs = thermo.liquid_spinodal(T, G)
    assert abs(thermo.dp_drho(rs, T, G)) < 1e-12
    assert math.isclose(rs, eos.spinodal(T, G)[1], rel_tol=1e-9)


def test_hydrostatic_column():
    n, rho, g = 64, 2.49, 2e-5
    T_d, T_u = 0.95 * TC, 0.85 * TC
    prof = thermo.hydrostatic_profile(n, rho, T_d, T_u, G, g)
    assert math.isclose(sum(prof) / n, rho, rel_tol=1e-9)
    T = [T_d + (T_u - T_d) * (k + 0.5) / n for k in range(n)]
    P = [thermo.pressure(r, t, G) for r, t in zip(prof, T)]
    for k in range(n - 1):   # trapezoidal hydrostatic balance between planes
        assert math.isclose(P[k + 1] - P[k], -0.5 * g * (prof[k] + prof[k + 1]), rel_tol=1e-6,
                            abs_tol=1e-12)
    # a boiling mean density has no liquid column (its bottom lies past the spinodal)
    thr = thermo.boiling_threshold_density(n, T_d, T_u, G, g)
    assert thermo.hydrostatic_profile(n, thr - 0.1, T_d, T_u, G, g) is None
