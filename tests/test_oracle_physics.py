"""Physics pins of the oracle: textbook closed forms its dynamics must meet.

Each test fails for a plausible mistake in a specific part of the oracle:
* shear-wave decay (periodic and between the walls): viscosity
  nu = (tau_nu - 1/2)/3 of the BGK f equation and the half-way position of
  the bounce-back walls;
* advection of an isobaric temperature mode by a uniform flow: the direction
  of streaming and the velocity in g^eq;
* sound speed: the ideal pressure rho T put into f^eq (f/g coupling) plus the
  counter-term of the g equation make sound adiabatic, c^2 = T (1 + 1/c_v),
  with T'/T = (1/c_v) rho'/rho (second form of eq. (eq)); without the
  counter-term sound is isothermal;
* entropy-mode decay: one conductivity kappa = c_v (tau_kappa - 1/2) rho_kappa
  / 3 in both phases (Table 1 uses one kappa for chi_l and chi_g); the
  isobaric mode decays at kappa k^2 / (rho c_p), c_p = c_v + 1;
* steady conduction between the walls with gravity: anti-bounce-back wall
  temperatures and the physical velocity v = (j + F/2)/rho give v_z = 0, a
  linear T(z) and Nu = 1 at both walls (eq. (flux) with no convection).
"""
import math

import numpy as np
import pytest
import torch

from oracle import lbm

DT = torch.float64
T0 = 0.05   # working temperature of the tests (the default critical temperature)


def _state(p, rho, u, T):
    f = lbm.f_equilibrium(rho, u, p.T_lattice)
    g = lbm.g_equilibrium(p, rho, rho * T, u, T)
    return f, g


def _run(p, f, g, n):
    with torch.no_grad():
        for _ in range(n):
            f, g = lbm.step(p, f, g)
    return f, g


def _shear_rate(tau, n=64, steps=(60, 560)):
    p = lbm.Params(1, n, 1, tau_nu=tau, tau_kappa=1.0, G=0.0, periodic_z=True)
    y = torch.arange(n, dtype=DT)
    k = 2 * math.pi / n
    rho = torch.ones(1, n, 1, dtype=DT)
    T = torch.full((1, n, 1), T0, dtype=DT)
    u = torch.zeros(3, 1, n, 1, dtype=DT)
    u[0, 0, :, 0] = 1e-4 * torch.sin(k * y)
    f, g = _state(p, rho, u, T)
    amps = []
    t = 0
    for s in steps:
        f, g = _run(p, f, g, s - t)
        t = s
        ux = lbm.macroscopic(p, f, g)["v"][0, 0, :, 0]
        amps.append((ux * torch.sin(k * y)).sum().item() * 2 / n)
    rate = -math.log(amps[1] / amps[0]) / (steps[1] - steps[0])
    return rate, p.nu * k * k


@pytest.mark.parametrize("tau", [0.6, 1.0, 1.4])
def test_shear_wave_viscosity(tau):
    rate, want = _shear_rate(tau)
    assert abs(rate / want - 1) < 5e-3


@pytest.mark.parametrize("tau", [0.8, 1.0])
def test_wall_bounded_shear_mode(tau):
    """Slowest Stokes mode between no-slip walls at z = -1/2 and H - 1/2:
    u_x = sin(pi (z + 1/2) / H) decays at nu (pi/H)^2."""
    H = 24
    p = lbm.Params(1, 1, H, tau_nu=tau, tau_kappa=1.0, G=0.0, T_d=T0, T_u=T0)
    z = torch.arange(H, dtype=DT)
    shape = torch.sin(math.pi * (z + 0.5) / H)
    rho = torch.ones(H, 1, 1, dtype=DT)
    T = torch.full((H, 1, 1), T0, dtype=DT)
    u = torch.zeros(3, H, 1, 1, dtype=DT)
    u[0, :, 0, 0] = 1e-4 * shape
    f, g = _state(p, rho, u, T)
    f, g = _run(p, f, g, 100)
    a0 = (lbm.macroscopic(p, f, g)["v"][0, :, 0, 0] * shape).sum().item()
    f, g = _run(p, f, g, 600)
    a1 = (lbm.macroscopic(p, f, g)["v"][0, :, 0, 0] * shape).sum().item()
    rate = -math.log(a1 / a0) / 600
    want = p.nu * (math.pi / H) ** 2
    assert abs(rate / want - 1) < 1e-2


def _isobaric_mode(p, n, rho0, T0, amp, U=0.0):
    x = torch.arange(n, dtype=DT)
    k = 2 * math.pi / n
    Tp = T0 * amp * torch.cos(k * x)
    T = (T0 + Tp).view(1, 1, n)
    rho = (rho0 - rho0 * Tp / T0).view(1, 1, n)
    u = torch.zeros(3, 1, 1, n, dtype=DT)
    u[0] = U
    return _state(p, rho, u, T), x, k


def _mode(field, x, k):
    c = (field * torch.cos(k * x)).sum().item()
    s = (field * torch.sin(k * x)).sum().item()
    return c, s


def test_advection_direction_and_speed():
    n, U = 64, 0.05
    p = lbm.Params(n, 1, 1, tau_nu=0.8, tau_kappa=1.0, G=0.0, periodic_z=True)
    (f, g), x, k = _isobaric_mode(p, n, 1.0, T0, 1e-3, U=U)
    steps = 300
    f, g = _run(p, f, g, steps)
    T = lbm.macroscopic(p, f, g)["T"].view(n)
    c, s = _mode(T - T.mean(), x, k)
    phase = math.atan2(s, c)          # cos(k(x - U t)) has phase +k U t
    assert abs(phase / (k * U * steps) - 1) < 0.02


@pytest.mark.parametrize("rho0,rho_kappa,tau_kappa", [(1.0, 0.5, 1.0), (1.0, 1.0, 1.0),
                                                      (2.0, 0.5, 1.0), (1.0, 0.5, 0.8)])
def test_entropy_mode_diffusivity(rho0, rho_kappa, tau_kappa):
    n = 32
    p = lbm.Params(n, 1, 1, tau_nu=1.0, tau_kappa=tau_kappa, G=0.0, rho_kappa=rho_kappa,
                   periodic_z=True)
    (f, g), x, k = _isobaric_mode(p, n, rho0, T0, 1e-3)
    want = p.kappa * k * k / (rho0 * (p.c_v + 1.0))
    t0 = int(1.0 / want)          # let the acoustic transient die out first
    f, g = _run(p, f, g, t0)
    a0 = _mode(lbm.macroscopic(p, f, g)["T"].view(n), x, k)[0]
    f, g = _run(p, f, g, 300)
    a1 = _mode(lbm.macroscopic(p, f, g)["T"].view(n), x, k)[0]
    rate = -math.log(a1 / a0) / 300
    assert abs(rate / want - 1) < 5e-2   # O(k^2) lattice correction ~3% at k = 2 pi / 32


@pytest.mark.parametrize("c_v", [1.0, 2.0])
def test_adiabatic_sound_speed(c_v):
    from scipy.optimize import curve_fit
    n = 64
    rho0, amp = 1.0, 1e-4
    p = lbm.Params(n, 1, 1, tau_nu=0.8, tau_kappa=0.6, G=0.0, c_v=c_v, periodic_z=True)
    x = torch.arange(n, dtype=DT)
    k = 2 * math.pi / n
    rp = amp * torch.cos(k * x)
    rho = (rho0 * (1 + rp)).view(1, 1, n)
    T = (T0 * (1 + rp / c_v)).view(1, 1, n)
    f, g = _state(p, rho, torch.zeros(3, 1, 1, n, dtype=DT), T)
    ts, ar, aT = [], [], []
    for t in range(0, 400):
        m = lbm.macroscopic(p, f, g)
        ts.append(t)
        ar.append(_mode(m["rho"].view(n), x, k)[0] * 2 / n / rho0)
        aT.append(_mode(m["T"].view(n), x, k)[0] * 2 / n / T0)
        f, g = _run(p, f, g, 1)
    ts, ar, aT = map(np.array, (ts, ar, aT))

    def model(t, A, gam, w, ph, B, d):
        return A * np.exp(-gam * t) * np.cos(w * t + ph) + B * np.exp(-d * t)

    c2 = T0 * (1 + 1 / c_v)
    w0 = math.sqrt(c2) * k
    popt, _ = curve_fit(model, ts, ar, p0=[amp, 1e-3, w0, 0.0, 0.0, 1e-4])
    assert abs(popt[2] / w0 - 1) < 5e-3
    # adiabatic temperature swing T'/T = (1/c_v) rho'/rho on the oscillating part
    poptT, _ = curve_fit(model, ts, aT, p0=[amp / c_v, 1e-3, w0, 0.0, 0.0, 1e-4])
    assert abs(poptT[0] / popt[0] * c_v - 1) < 2e-2


def test_steady_conduction_nusselt_one():
    """Single-phase ideal gas between walls with gravity: the steady state
    is at rest (v_z = 0), T(z) is linear and Nu = 1 at both walls and in the
    bulk."""
    nz = 8
    p = lbm.Params(2, 2, nz, tau_nu=1.0, tau_kappa=1.5, G=0.0, T_d=0.048, T_u=0.042,
                   gravity=1e-3)
    rho0 = torch.ones(nz, 2, 2, dtype=DT)
    f, g = lbm.init_state(p, rho0)
    f, g = _run(p, f, g, 3000)
    nu_bot, nu_top, nu_z, Tz = lbm.nusselt(p, f, g)
    m = lbm.macroscopic(p, f, g)
    assert m["v"].abs().max() < 1e-12
    assert abs(nu_bot.item() - 1) < 1e-10 and abs(nu_top.item() - 1) < 1e-10
    assert (nu_z - 1).abs().max() < 1e-10
    kk = torch.arange(nz, dtype=DT)
    lin = p.T_d + (p.T_u - p.T_d) * (kk + 0.5) / nz
    assert (Tz - lin).abs().max() < 1e-12
    # wall heat flux of the conductive state: kappa (T_d - T_u) / H
    q = lbm.q_bottom(p, f, g).item()
    assert abs(q / (p.kappa * (p.T_d - p.T_u) / nz) - 1) < 1e-10
    # hydrostatic stratification is really there (density increases downwards)
    rz = m["rho"].mean(dim=(1, 2))
    assert rz[0] > rz[-1]
