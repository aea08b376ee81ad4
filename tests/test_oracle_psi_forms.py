"""Pins of the oracle's alternative pseudopotential, the original Shan-Chen
psi = 1 - exp(-rho) (one of the forms the paper cites as prior art before
fixing psi = exp(-1/rho) for thermodynamic consistency), on the CPU.

* EOS P = rho T + (G/2) psi^2: critical point at rho_c = ln 2, T_c = -G/4
  (first and second density derivatives of P vanish there);
* bulk force: on a smooth density field the stencil force tends to
  -(G/2) grad psi^2 = -G psi psi' grad rho (second order in k);
* coexistence of a flat interface at uniform temperature (the lattice
  temperature of f^eq equal to T, so the thermal force vanishes): the liquid
  density within 0.3 % and the vapour density within 4 % of the
  mechanical-stability rule of this psi (area weight psi'/psi), and the
  liquid more than 1 % off the Maxwell construction (weight 1/rho^2), which
  this psi does not satisfy;
* a wetting wall uses psi of the wall density in the same form.
"""
import math

import pytest
import torch

from oracle import eos, lbm

DT = torch.float64
G_SC = -0.2          # T_c = 0.05


def test_critical_point_of_the_sc_eos():
    rc, tc = eos.critical_point_sc(G_SC)
    assert abs(tc - 0.05) < 1e-15
    h = 1e-5
    d1 = (eos.pressure_sc(rc + h, tc, G_SC) - eos.pressure_sc(rc - h, tc, G_SC)) / (2 * h)
    d2 = (eos.pressure_sc(rc + h, tc, G_SC) - 2 * eos.pressure_sc(rc, tc, G_SC)
          + eos.pressure_sc(rc - h, tc, G_SC)) / (h * h)
    assert abs(d1) < 1e-10 and abs(d2) < 1e-5
    assert abs(eos.dp_drho_sc(rc, tc, G_SC)) < 1e-15
    # below T_c the isotherm has a loop
    assert eos.dp_drho_sc(rc, 0.9 * tc, G_SC) < 0


def test_sc_force_matches_eos_gradient():
    n = 256
    p = lbm.Params(1, 1, n, G=G_SC, periodic_z=True, psi_form=1)
    z = torch.arange(n, dtype=DT)
    k = 2 * torch.pi / n
    rho = (1.0 + 0.3 * torch.sin(k * z)).view(n, 1, 1)
    F = lbm.sc_force(p, rho)
    r = rho.view(n)
    drho = 0.3 * k * torch.cos(k * z)
    want = -G_SC * (1.0 - torch.exp(-r)) * torch.exp(-r) * drho
    err = (F[2].view(n) - want).abs().max() / want.abs().max()
    assert err < 2e-3
    assert F[0].abs().max() < 1e-15 and F[1].abs().max() < 1e-15
    # and the paper's form is not what this gives
    p0 = p.with_(psi_form=0)
    assert (lbm.sc_force(p0, rho)[2].view(n) - want).abs().max() / want.abs().max() > 0.1


def _slab(t, nz=96, steps=3000):
    T = t * 0.05
    rg, rl, _ = eos.coexistence_sc(T, G_SC)
    p = lbm.Params(1, 1, nz, tau_nu=1.0, tau_kappa=1.5, G=G_SC, c_v=10.0, T_lat=T, T_d=T, T_u=T,
                   periodic_z=True, psi_form=1)
    z = torch.arange(nz, dtype=DT)
    prof = rg + (rl - rg) * 0.5 * (torch.tanh((z - nz / 4) / 3) - torch.tanh((z - 3 * nz / 4) / 3))
    f, g = lbm.init_state(p, prof.view(nz, 1, 1), torch.full((nz, 1, 1), T, dtype=DT))
    with torch.no_grad():
        for _ in range(steps):
            f, g = lbm.step(p, f, g)
    r = lbm.macroscopic(p, f, g)["rho"].view(nz)
    return r[0].item(), r[nz // 2].item(), T


@pytest.mark.slow
@pytest.mark.parametrize("t", [0.85, 0.9])
def test_sc_flat_interface_on_its_mechanical_rule(t):
    rho_g, rho_l, T = _slab(t)
    mg, ml, _ = eos.coexistence_sc(T, G_SC)
    xg, xl, _ = eos.coexistence_sc(T, G_SC, rule="maxwell")
    assert abs(rho_l / ml - 1) < 3e-3, (rho_l, ml)
    assert abs(rho_g / mg - 1) < 4e-2, (rho_g, mg)
    assert abs(rho_l / xl - 1) > 1e-2, (rho_l, xl)
    assert abs(rho_g / mg - 1) < 0.5 * abs(rho_g / xg - 1)


def test_sc_wall_ghost():
    rho0, rw = 1.2, 2.0
    p = lbm.Params(3, 4, 6, G=G_SC, rho_wall_d=rw, psi_form=1)
    F = lbm.sc_force(p, torch.full((6, 4, 3), rho0, dtype=DT))
    psi = 1.0 - math.exp(-rho0)
    want = 0.5 * G_SC * psi * ((1.0 - math.exp(-rw)) - psi)
    assert float((F[2, 0] - want).abs().max()) < 1e-15
