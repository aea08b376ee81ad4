"""Pins of the oracle's wetting walls (a prescribed wall density for the psi
ghost plane; the paper is silent on wettability, this is the wall-density
method of Benzi et al., Phys. Rev. E 74, 021509 (2006)), on the CPU.

* a wall density equal to that of a uniform fluid is the neutral (mirror)
  wall: no force anywhere;
* the Shan-Chen force on a uniform fluid next to a wall of density rho_w has
  the closed form F_z = +-(G/2) psi(rho) (psi(rho_w) - psi(rho)) on the wall
  plane (the five directions that cross the wall carry sum W c_z = -+1/2)
  and vanishes elsewhere;
* a 1-D column at 0.8 T_c, started uniform at the mean of the coexistence
  densities: walls of vapour density end with vapour against both walls
  and liquid in the middle; walls of liquid density keep liquid against the
  walls.
"""
import math

import torch

from oracle import eos, lbm

DT = torch.float64
TC = 0.05
G = eos.coupling_for_tc(TC)


def _uniform(n, rho):
    return torch.full((n, 4, 3), rho, dtype=DT)


def test_wall_density_of_a_uniform_fluid_is_neutral():
    rho0 = 1.7
    p = lbm.Params(3, 4, 9, G=G, rho_wall_d=rho0, rho_wall_u=rho0)
    F = lbm.sc_force(p, _uniform(9, rho0))
    F_mirror = lbm.sc_force(p.with_(rho_wall_d=0.0, rho_wall_u=0.0), _uniform(9, rho0))
    assert float(F.abs().max()) < 1e-16
    assert float(F_mirror.abs().max()) < 1e-16


def test_first_layer_force_closed_form():
    rho0, rwd, rwu = 1.5, 2.2, 0.6
    nz = 7
    p = lbm.Params(3, 4, nz, G=G, rho_wall_d=rwd, rho_wall_u=rwu)
    F = lbm.sc_force(p, _uniform(nz, rho0))
    psi = math.exp(-1.0 / rho0)
    want_d = 0.5 * G * psi * (math.exp(-1.0 / rwd) - psi)
    want_u = -0.5 * G * psi * (math.exp(-1.0 / rwu) - psi)
    scale = abs(want_d) + abs(want_u)
    assert float(F[:2].abs().max()) < 1e-15 * scale          # no horizontal force
    assert float((F[2, 0] - want_d).abs().max()) < 1e-14 * scale
    assert float((F[2, -1] - want_u).abs().max()) < 1e-14 * scale
    assert float(F[2, 1:-1].abs().max()) < 1e-15 * scale     # interior untouched
    # an attracting (denser) bottom wall pulls the fluid down
    assert want_d < 0


def _column(rho_w, nz=48, steps=3000):
    T = 0.8 * TC
    rg, rl, _ = eos.maxwell(T, G)
    p = lbm.Params(1, 1, nz, tau_nu=1.0, tau_kappa=1.5, G=G, c_v=10.0, T_lat=T, T_d=T, T_u=T,
                   rho_wall_d=rho_w(rg, rl), rho_wall_u=rho_w(rg, rl))
    f, g = lbm.init_state(p, torch.full((nz, 1, 1), 0.5 * (rg + rl), dtype=DT),
                          torch.full((nz, 1, 1), T, dtype=DT))
    with torch.no_grad():
        for _ in range(steps):
            f, g = lbm.step(p, f, g)
    return lbm.macroscopic(p, f, g)["rho"].view(nz), rg, rl


def test_vapour_walls_dry_and_liquid_walls_wet():
    r, rg, rl = _column(lambda rg, rl: rg)
    nz = r.numel()
    for k in (0, nz - 1):
        assert abs(r[k].item() / rg - 1) < 0.05, r[k].item()
    assert abs(r[nz // 2].item() / rl - 1) < 0.05, r[nz // 2].item()
    r, rg, rl = _column(lambda rg, rl: rl)
    for k in (0, nz - 1):
        assert abs(r[k].item() / rl - 1) < 0.05, r[k].item()
