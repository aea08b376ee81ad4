"""Thermodynamic pins of the oracle's pseudopotential + thermal coupling
(Fig. 1: Clausius-Clapeyron check; Laplace's law), on the CPU.

* flat interface at uniform temperature (periodic z, 1-D): bulk densities
  within 2 % of the Maxwell construction of the model's EOS, equal bulk
  pressures (mechanical balance) and one temperature in both phases;
* Clausius-Clapeyron (Fig. 1): the slope of the measured coexistence
  pressure P_sat(T) between 0.75 and 0.85 T_c against
  Delta s / Delta v = ln(rho_l/rho_g) / (1/rho_g - 1/rho_l) at 0.8 T_c
  (measured densities), within 4 %;
* Laplace: cylindrical drops of three radii at uniform temperature; the
  pressure jump is linear in 1/R with a positive surface tension and an
  intercept below 10 % of the largest jump.
"""
import math

import pytest
import torch

from oracle import eos, lbm

DT = torch.float64
TC = 0.05
G = eos.coupling_for_tc(TC)

pytestmark = pytest.mark.slow


def _slab(t, nz=96, steps=3000):
    # a large c_v keeps the latent heat of the initial relaxation from
    # shifting the temperature; the EOS does not depend on c_v
    T = t * TC
    rg, rl, _ = eos.maxwell(T, G)
    p = lbm.Params(1, 1, nz, tau_nu=1.0, tau_kappa=1.5, G=G, c_v=10.0, T_lat=0.8 * TC,
                   periodic_z=True)
    z = torch.arange(nz, dtype=DT)
    prof = rg + (rl - rg) * 0.5 * (torch.tanh((z - nz / 4) / 3) - torch.tanh((z - 3 * nz / 4) / 3))
    f, g = lbm.init_state(p, prof.view(nz, 1, 1), torch.full((nz, 1, 1), T, dtype=DT))
    with torch.no_grad():
        for _ in range(steps):
            f, g = lbm.step(p, f, g)
    m = lbm.macroscopic(p, f, g)
    r, Tz = m["rho"].view(nz), m["T"].view(nz)
    return dict(rho_g=r[0].item(), rho_l=r[nz // 2].item(), T_g=Tz[0].item(), T_l=Tz[nz // 2].item())


@pytest.fixture(scope="module")
def slabs():
    return {t: _slab(t) for t in (0.75, 0.8, 0.85)}


@pytest.mark.parametrize("t", [0.75, 0.8, 0.85])
def test_flat_interface_against_maxwell(slabs, t):
    s = slabs[t]
    T = 0.5 * (s["T_g"] + s["T_l"])
    assert abs(s["T_l"] - s["T_g"]) / T < 1e-3
    rg, rl, P = eos.maxwell(T, G)
    assert abs(s["rho_g"] / rg - 1) < 0.02
    assert abs(s["rho_l"] / rl - 1) < 0.02
    Pg = eos.pressure(s["rho_g"], s["T_g"], G)
    Pl = eos.pressure(s["rho_l"], s["T_l"], G)
    assert abs(Pl - Pg) / P < 5e-3


def test_clausius_clapeyron(slabs):
    def psat(s):
        return 0.5 * (eos.pressure(s["rho_g"], s["T_g"], G) + eos.pressure(s["rho_l"], s["T_l"], G))

    def tmean(s):
        return 0.5 * (s["T_g"] + s["T_l"])

    lo, mid, hi = slabs[0.75], slabs[0.8], slabs[0.85]
    slope = (psat(hi) - psat(lo)) / (tmean(hi) - tmean(lo))
    want = eos.clausius_clapeyron_slope(mid["rho_g"], mid["rho_l"])
    assert abs(slope / want - 1) < 0.04


def _drop(R, n=56, steps=2000):
    T = 0.8 * TC
    rg, rl, _ = eos.maxwell(T, G)
    p = lbm.Params(n, n, 1, tau_nu=1.0, tau_kappa=1.5, G=G, c_v=10.0, T_lat=T, periodic_z=True)
    y, x = torch.meshgrid(torch.arange(n, dtype=DT), torch.arange(n, dtype=DT), indexing="ij")
    r = torch.sqrt((x - n / 2 + 0.5) ** 2 + (y - n / 2 + 0.5) ** 2)
    rho = rg + (rl - rg) * 0.5 * (1 - torch.tanh((r - R) / 2))
    f, g = lbm.init_state(p, rho.view(1, n, n), torch.full((1, n, n), T, dtype=DT))
    with torch.no_grad():
        for _ in range(steps):
            f, g = lbm.step(p, f, g)
    m = lbm.macroscopic(p, f, g)
    rho, Tf = m["rho"].view(n, n), m["T"].view(n, n)
    c = n // 2
    r_in, T_in = rho[c, c].item(), Tf[c, c].item()
    r_out, T_out = rho[0, 0].item(), Tf[0, 0].item()
    dP = eos.pressure(r_in, T_in, G) - eos.pressure(r_out, T_out, G)
    # equivalent radius from the liquid volume
    area = ((rho - r_out) / (r_in - r_out)).sum().item()
    return math.sqrt(area / math.pi), dP


def test_laplace_law_for_cylinders():
    pts = [_drop(R) for R in (10.0, 14.0, 18.0)]
    inv = [1.0 / R for R, _ in pts]
    dP = [d for _, d in pts]
    n = len(pts)
    mx, my = sum(inv) / n, sum(dP) / n
    sxx = sum((a - mx) ** 2 for a in inv)
    sxy = sum((a - mx) * (b - my) for a, b in zip(inv, dP))
    sigma = sxy / sxx
    icpt = my - sigma * mx
    assert sigma > 0
    assert abs(icpt) < 0.1 * max(dP)
    resid = max(abs(b - (icpt + sigma * a)) for a, b in zip(inv, dP))
    assert resid < 0.05 * max(dP)
