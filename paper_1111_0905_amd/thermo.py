"""Thermodynamics of the model's equation of state, for setting up runs.

P = rho T + (G/2) exp(-2/rho) (text after eq. (ns), with the factor 1/2 of
eq. (FORCE) written out); critical point rho_c = 1, T_c = -G/e^2.  Per unit
mass: (dP/dT)_rho = rho, so c_p - c_v = T / (dP/drho)_T and the isobaric
expansion coefficient is beta = 1 / (dP/drho)_T.  Transport: nu =
(tau_nu - 1/2)/3, kappa = c_v (tau_kappa - 1/2) rho_kappa / 3,
chi = kappa / (rho c_p).  Rayleigh number as in the caption of Table 1:
Ra = g beta L^4 (Delta T / L - gamma_ad) / (chi nu), gamma_ad = beta T g / c_p.
"""
from __future__ import annotations

import math


def coupling_for_tc(T_c: float) -> float:
    return -T_c * math.e ** 2


def pressure(rho: float, T: float, G: float) -> float:
    return rho * T + 0.5 * G * math.exp(-2.0 / rho)


def dp_drho(rho: float, T: float, G: float) -> float:
    return T + G * math.exp(-2.0 / rho) / (rho * rho)


def cp(rho: float, T: float, G: float, c_v: float = 1.0) -> float:
    return c_v + T / dp_drho(rho, T, G)


def beta(rho: float, T: float, G: float) -> float:
    return 1.0 / dp_drho(rho, T, G)


def kappa(tau_kappa: float, rho_kappa: float, c_v: float = 1.0) -> float:
    return c_v * (tau_kappa - 0.5) * rho_kappa / 3.0


def tau_kappa_for_prandtl(Pr: float, nu: float, rho: float, T: float, G: float,
                          rho_kappa: float = 0.5, c_v: float = 1.0) -> float:
    """tau_kappa giving Pr = nu / chi in a phase of density rho at T."""
    k = nu / Pr * rho * cp(rho, T, G, c_v)
    return 0.5 + 3.0 * k / (c_v * rho_kappa)


def _ra_coefficients(L, rho, T_d, T_u, G, tau_nu, tau_kappa, rho_kappa, c_v):
    # Ra chi nu = g b L^3 dT - g^2 b^2 T L^4 / c  ->  A g^2 + B g + C(Ra) = 0
    T = 0.5 * (T_d + T_u)
    b, c = beta(rho, T, G), cp(rho, T, G, c_v)
    chi = kappa(tau_kappa, rho_kappa, c_v) / (rho * c)
    nu = (tau_nu - 0.5) / 3.0
    return b * b * T * L ** 4 / c, -b * L ** 3 * (T_d - T_u), chi * nu


def max_rayleigh(L, rho, T_d, T_u, G, tau_nu, tau_kappa, rho_kappa=0.5, c_v=1.0) -> float:
    """Largest Ra any gravity reaches (the adiabatic gradient grows with g)."""
    A, B, cn = _ra_coefficients(L, rho, T_d, T_u, G, tau_nu, tau_kappa, rho_kappa, c_v)
    return B * B / (4 * A * cn)


def gravity_for_rayleigh(Ra: float, L: int, rho: float, T_d: float, T_u: float, G: float,
                         tau_nu: float, tau_kappa: float, rho_kappa: float = 0.5,
                         c_v: float = 1.0) -> float:
    """Smallest g with Ra(g) = Ra at the mid temperature and density rho."""
    A, B, cn = _ra_coefficients(L, rho, T_d, T_u, G, tau_nu, tau_kappa, rho_kappa, c_v)
    disc = B * B - 4 * A * Ra * cn
    if disc < 0:
        raise ValueError("Rayleigh number not reachable: the adiabatic gradient dominates "
                         f"(max Ra {B * B / (4 * A * cn):.3g})")
    return (-B - math.sqrt(disc)) / (2 * A)


def liquid_spinodal(T: float, G: float) -> float:
    """Density above 1 where (dP/drho)_T = 0 (the metastable liquid's end)."""
    lo, hi = 1.0, 50.0
    for _ in range(64):
        mid = 0.5 * (lo + hi)
        if dp_drho(mid, T, G) < 0:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def liquid_density(P: float, T: float, G: float, spinodal: float = None) -> float:
    """rho on the liquid branch with P(rho, T) = P; nan when P is below the
    spinodal pressure (no liquid state exists)."""
    lo = liquid_spinodal(T, G) if spinodal is None else spinodal
    if pressure(lo, T, G) > P:
        return float("nan")
    hi = lo + 1.0
    while pressure(hi, T, G) < P:
        hi *= 2.0
    for _ in range(64):
        mid = 0.5 * (lo + hi)
        if pressure(mid, T, G) < P:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def liquid_column(P_bottom: float, n: int, T_d: float, T_u: float, G: float, g: float):
    """Hydrostatic liquid column on the n node planes of the cell: node k at
    height k + 1/2 with the conduction temperature T_d + (T_u - T_d)(k + 1/2)/n;
    dP/dz = -rho g by the trapezoidal rule, rho on the liquid branch."""
    T = [T_d + (T_u - T_d) * (k + 0.5) / n for k in range(n)]
    P = P_bottom
    rho = [liquid_density(P, T[0], G)]
    for k in range(1, n):
        r = rho[-1]
        sp = liquid_spinodal(T[k], G)
        for _ in range(4):
            r = liquid_density(P - 0.5 * g * (rho[-1] + r), T[k], G, sp)
        P -= 0.5 * g * (rho[-1] + r)
        rho.append(r)
    return rho


def boiling_threshold_density(n: int, T_d: float, T_u: float, G: float, g: float) -> float:
    """Mean density of the hydrostatic liquid column whose bottom node sits on
    the liquid spinodal: a lower mean density puts the bottom layer inside the
    unstable region, where vapour nucleates."""
    T0 = T_d + (T_u - T_d) * 0.5 / n
    rs = liquid_spinodal(T0, G)
    rho = liquid_column(pressure(rs, T0, G) + 1e-15, n, T_d, T_u, G, g)
    return sum(rho) / n


def hydrostatic_profile(n: int, rho_mean: float, T_d: float, T_u: float, G: float, g: float):
    """Liquid column of mean density rho_mean in hydrostatic balance on the
    conduction temperature profile (liquid_column with the bottom pressure
    found by bisection); None when some plane would have no liquid state."""
    T0 = T_d + (T_u - T_d) * 0.5 / n
    lo = pressure(liquid_spinodal(T0, G), T0, G) + 1e-15
    def mean_at(Pb):
        r = liquid_column(Pb, n, T_d, T_u, G, g)
        return sum(r) / n if all(x == x for x in r) else float("nan")
    m_lo = mean_at(lo)
    if not (m_lo == m_lo) or m_lo > rho_mean:
        return None
    hi = lo + 1.0
    while mean_at(hi) < rho_mean:
        hi = lo + 2.0 * (hi - lo)
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        if mean_at(mid) < rho_mean:
            lo = mid
        else:
            hi = mid
    return liquid_column(0.5 * (lo + hi), n, T_d, T_u, G, g)
