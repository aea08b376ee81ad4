"""Equation of state of the model and its coexistence curve (FP64, CPU).

TEST INFRASTRUCTURE ONLY (see oracle/lbm.py).

The paper's EOS (text after eq. (ns)) is P = P0 + P_NI with the ideal part
P0 = rho T and a non-ideal part exp(-2/rho) times the interaction strength.
With force weights normalised to sum W c c = 1, a Taylor expansion of
eq. (FORCE) gives F = -(G/2) grad psi^2, i.e. P_NI = (G/2) exp(-2/rho); the
paper's "G exp(-2/rho)" absorbs the factor 1/2.  Then
  dP/drho = T + G exp(-2/rho) / rho^2,  d2P/drho2 = 0 at rho = 1,
so rho_c = 1, T_c = -G/e^2 and P_c = T_c / 2.

Coexistence (Fig. 1): the Maxwell equal-area construction in the specific
volume v = 1/rho, P(rho_g) = P(rho_l) = P_sat and
  integral_{rho_g}^{rho_l} (P_sat - P(rho)) / rho^2 d rho = 0.
Entropy per unit mass of this model is s = c_v ln T - ln rho (the non-ideal
part carries no T dependence), so Delta s = ln(rho_l / rho_g) and the
Clausius-Clapeyron slope is dP_sat/dT = ln(rho_l/rho_g) / (1/rho_g - 1/rho_l).
"""
from __future__ import annotations

import math

from scipy.integrate import quad
from scipy.optimize import brentq


def pressure(rho: float, T: float, G: float) -> float:
    return rho * T + 0.5 * G * math.exp(-2.0 / rho)


def dp_drho(rho: float, T: float, G: float) -> float:
    return T + G * math.exp(-2.0 / rho) / (rho * rho)


def critical_temperature(G: float) -> float:
    return -G / math.e ** 2


def coupling_for_tc(T_c: float) -> float:
    return -T_c * math.e ** 2


def spinodal(T: float, G: float):
    """Densities where dP/drho = 0 (gas-side, liquid-side); T < T_c."""
    tc = critical_temperature(G)
    if not T < tc:
        raise ValueError("spinodal exists only below T_c")
    return (brentq(dp_drho, 0.05, 1.0, args=(T, G), xtol=1e-15),
            brentq(dp_drho, 1.0, 50.0, args=(T, G), xtol=1e-15))


def _density_at_pressure(P: float, T: float, G: float, lo: float, hi: float) -> float:
    return brentq(lambda r: pressure(r, T, G) - P, lo, hi, xtol=1e-15, rtol=1e-15)


def maxwell(T: float, G: float, weight=None):
    """(rho_g, rho_l, P_sat) of the equal-area construction.

    weight(rho) is the measure of the area rule; the default 1/rho^2 is
    Maxwell's.  Other weights give the mechanical-stability rules of
    pseudopotential models (used only for comparison in tests).
    """
    wfun = weight or (lambda r: 1.0 / (r * r))
    sg, sl = spinodal(T, G)
    p_lo = max(pressure(sl, T, G), 1e-12)
    p_hi = pressure(sg, T, G)

    def area(P):
        rg = _density_at_pressure(P, T, G, 1e-3, sg)
        rl = _density_at_pressure(P, T, G, sl, 200.0)
        val, _ = quad(lambda r: (P - pressure(r, T, G)) * wfun(r), rg, rl,
                      epsabs=1e-14, epsrel=1e-13, limit=200)
        return val

    P = brentq(area, p_lo * (1 + 1e-12), p_hi * (1 - 1e-12), xtol=1e-15, rtol=1e-14)
    rg = _density_at_pressure(P, T, G, 1e-3, sg)
    rl = _density_at_pressure(P, T, G, sl, 200.0)
    return rg, rl, P


def clausius_clapeyron_slope(rho_g: float, rho_l: float) -> float:
    """Delta s / Delta v for this model: ln(rho_l/rho_g) / (1/rho_g - 1/rho_l)."""
    return math.log(rho_l / rho_g) / (1.0 / rho_g - 1.0 / rho_l)


def latent_heat(T: float, rho_g: float, rho_l: float) -> float:
    """lambda = T Delta s (Fig. 1 inset)."""
    return T * math.log(rho_l / rho_g)


def nonideal_energy(rho: float, G: float) -> float:
    """integral of P_NI / rho^2 d rho with P_NI = (G/2) exp(-2/rho)."""
    return 0.25 * G * math.exp(-2.0 / rho)


# ---------------------------------------------------------------- psi forms

def psi_sc(rho: float) -> float:
    """The original Shan-Chen pseudopotential 1 - exp(-rho)."""
    return 1.0 - math.exp(-rho)


def pressure_sc(rho: float, T: float, G: float) -> float:
    """Bulk EOS with psi = 1 - exp(-rho): P = rho T + (G/2) psi^2."""
    return rho * T + 0.5 * G * psi_sc(rho) ** 2


def dp_drho_sc(rho: float, T: float, G: float) -> float:
    return T + G * psi_sc(rho) * math.exp(-rho)


def critical_point_sc(G: float):
    """d2P/drho2 = G exp(-rho) (2 exp(-rho) - 1) = 0 at rho_c = ln 2, where
    dP/drho = 0 gives T_c = -G/4.  Returns (rho_c, T_c)."""
    return math.log(2.0), -G / 4.0


def coexistence_sc(T: float, G: float, rule: str = "mechanical"):
    """(rho_g, rho_l, P) of the psi = 1 - exp(-rho) fluid at temperature T:
    equal pressures and a zero area integral_{rho_g}^{rho_l} (P - P(rho)) w(rho)
    d rho, with w = psi'/psi (the mechanical-stability rule of a
    pseudopotential fluid whose forcing stencil adds no correction, which
    for psi = exp(-1/rho) is Maxwell's 1/rho^2) or, with rule "maxwell",
    w = 1/rho^2."""
    if rule == "mechanical":
        w = lambda r: math.exp(-r) / psi_sc(r)
    else:
        w = lambda r: 1.0 / (r * r)
    rc, tc = critical_point_sc(G)
    if not T < tc:
        raise ValueError("no coexistence above T_c")
    sg = brentq(dp_drho_sc, 1e-6, rc, args=(T, G), xtol=1e-15)
    sl = brentq(dp_drho_sc, rc, 50.0, args=(T, G), xtol=1e-15)
    p_lo = max(pressure_sc(sl, T, G), 1e-14)
    p_hi = pressure_sc(sg, T, G)

    def dens(P, lo, hi):
        return brentq(lambda r: pressure_sc(r, T, G) - P, lo, hi, xtol=1e-15, rtol=1e-15)

    def area(P):
        rg, rl = dens(P, 0.0, sg), dens(P, sl, 200.0)
        val, _ = quad(lambda r: (P - pressure_sc(r, T, G)) * w(r), rg, rl,
                      epsabs=1e-14, epsrel=1e-13, limit=200)
        return val

    P = brentq(area, p_lo * (1 + 1e-12), p_hi * (1 - 1e-12), xtol=1e-16, rtol=1e-14)
    return dens(P, 0.0, sg), dens(P, sl, 200.0), P
