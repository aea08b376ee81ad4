"""Pins of the equation-of-state helpers (text after eq. (ns), Fig. 1).

* critical point: with P = rho T + (G/2) exp(-2/rho), dP/drho and d2P/drho2
  vanish together at rho = 1, T = -G/e^2 (checked by finite differences);
* Maxwell coexistence: the Clausius-Clapeyron identity of Fig. 1,
  dP_sat/dT = Delta s / Delta v, holds for the computed binodal (finite
  difference of P_sat(T) against ln(rho_l/rho_g)/(1/rho_g - 1/rho_l)); a
  wrong area weight breaks it;
* internal energy: the non-ideal part of U equals the integral of
  P_NI / rho^2 (quadrature);
* Table 1 consistency of one conductivity: chi_g / chi_l = 0.008/0.0018 is
  matched by c_p rho ratios of this EOS near 0.9 T_c with c_v = 1.
"""
import json
import math
import os

import pytest
from scipy.integrate import quad

from oracle import eos

G = eos.coupling_for_tc(0.05)
TC = eos.critical_temperature(G)
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_critical_point():
    h = 1e-4
    d1 = (eos.pressure(1 + h, TC, G) - eos.pressure(1 - h, TC, G)) / (2 * h)
    d2 = (eos.pressure(1 + h, TC, G) - 2 * eos.pressure(1, TC, G) + eos.pressure(1 - h, TC, G)) / h ** 2
    assert abs(d1) < 1e-9 and abs(d2) < 1e-6
    assert abs(eos.pressure(1, TC, G) - TC / 2) < 1e-15


@pytest.mark.parametrize("t", [0.8, 0.85, 0.9, 0.95])
def test_maxwell_satisfies_clausius_clapeyron(t):
    T = t * TC
    h = 1e-5 * TC
    pp = eos.maxwell(T + h, G)[2]
    pm = eos.maxwell(T - h, G)[2]
    rg, rl, P = eos.maxwell(T, G)
    assert abs(eos.pressure(rg, T, G) - eos.pressure(rl, T, G)) < 1e-13
    slope = (pp - pm) / (2 * h)
    assert abs(slope / eos.clausius_clapeyron_slope(rg, rl) - 1) < 1e-6


def test_wrong_area_weight_breaks_clausius_clapeyron():
    T = 0.9 * TC
    h = 1e-5 * TC
    wrong = lambda r: 1.0 / r  # noqa: E731
    pp = eos.maxwell(T + h, G, weight=wrong)[2]
    pm = eos.maxwell(T - h, G, weight=wrong)[2]
    rg, rl, _ = eos.maxwell(T, G, weight=wrong)
    assert abs((pp - pm) / (2 * h) / eos.clausius_clapeyron_slope(rg, rl) - 1) > 1e-2


def test_nonideal_energy_is_integral():
    for rho in [0.3, 0.9, 1.7, 2.5]:
        val, _ = quad(lambda r: 0.5 * G * math.exp(-2 / r) / r ** 2, 1e-3, rho, epsabs=1e-15)
        assert abs(val - eos.nonideal_energy(rho, G)) < 1e-12


def test_oracle_internal_energy_matches_eos():
    import torch
    from oracle import lbm
    p = lbm.Params(1, 1, 1, G=G, c_v=1.5)
    for rho, T in [(0.5, 0.04), (1.9, 0.047)]:
        U = lbm.internal_energy(p, torch.tensor(rho, dtype=torch.float64), torch.tensor(T, dtype=torch.float64))
        assert abs(U.item() - (1.5 * T + eos.nonideal_energy(rho, G))) < 1e-15


def test_table1_diffusivity_ratio_one_conductivity():
    with open(os.path.join(GOLDEN, "table1.json")) as fh:
        tab = json.load(fh)
    ratio = tab["BOILING"]["chi_g"] / tab["BOILING"]["chi_l"]
    T = 0.9 * TC
    rg, rl, _ = eos.maxwell(T, G)
    cp = lambda r: 1.0 + T / eos.dp_drho(r, T, G)  # noqa: E731  (c_v = 1)
    predicted = cp(rl) * rl / (cp(rg) * rg)   # chi = kappa / (c_p rho) with one kappa
    assert abs(predicted / ratio - 1) < 0.02
    # the same ratio with kappa proportional to rho would be far off
    assert abs(cp(rl) / cp(rg) / ratio - 1) > 0.5
