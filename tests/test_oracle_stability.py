"""Linear stability of the oracle step at the paper's parameters.

The paper runs the scheme at nu = 0.0165 (tau_nu = 0.5495, Table 1) for long
times at 512^3, so its discrete dynamics is stable there.  A reading of the
unprinted equilibria must be too: the spectral radius of the one-step
Jacobian around every uniform rest state, per horizontal wavenumber, must not
exceed 1.  Autograd of the torch oracle gives the Jacobian.
"""
import numpy as np
import pytest
import torch

from oracle import eos, lbm

DT = torch.float64


def _spectral_radii(p, T0, rho0):
    n = p.nx
    shape = (1, 1, n)
    f, g = lbm.init_state(p, torch.full(shape, rho0, dtype=DT), torch.full(shape, T0, dtype=DT))
    s0 = torch.cat([f, g]).reshape(-1)

    def fn(s):
        s = s.view(38, *shape)
        a, b = lbm.step(p, s[:19], s[19:])
        return torch.cat([a, b]).reshape(-1)

    J = torch.autograd.functional.jacobian(fn, s0, vectorize=True).numpy().reshape(38, n, 38, n)
    out = []
    for m in range(n // 2 + 1):
        B = sum(J[:, x, :, 0] * np.exp(-2j * np.pi * m * x / n) for x in range(n))
        out.append(np.abs(np.linalg.eigvals(B)).max())
    return out


@pytest.mark.parametrize("taus", [(0.5495, 0.6417), (1.0, 1.0)])
@pytest.mark.parametrize("state", [(0.9, 0.55), (0.9, 1.8), (0.97, 2.0)])
def test_stable_around_rest_states(taus, state):
    Tc = 0.05
    p = lbm.Params(8, 1, 1, tau_nu=taus[0], tau_kappa=taus[1], G=eos.coupling_for_tc(Tc),
                   periodic_z=True)
    radii = _spectral_radii(p, state[0] * Tc, state[1])
    assert max(radii) < 1 + 1e-9
    # the conserved modes sit exactly on the unit circle at k = 0
    assert abs(radii[0] - 1) < 1e-9


def _walled_column_radius(Tc, rho, n=24, taus=(0.5495, 0.5947)):
    """Largest |eigenvalue| of the one-step Jacobian of a 1 x 1 x n column
    between two isothermal walls, about the uniform rest state."""
    Tm = 0.9 * Tc
    p = lbm.Params(1, 1, n, tau_nu=taus[0], tau_kappa=taus[1], G=eos.coupling_for_tc(Tc),
                   T_lat=Tm, T_d=Tm, T_u=Tm)
    shape = (n, 1, 1)
    f, g = lbm.init_state(p, torch.full(shape, rho, dtype=DT), torch.full(shape, Tm, dtype=DT))
    s0 = torch.cat([f, g]).reshape(-1)

    def fn(s):
        s = s.view(38, *shape)
        a, b = lbm.step(p, s[:19], s[19:])
        return torch.cat([a, b]).reshape(-1)

    J = torch.autograd.functional.jacobian(fn, s0, vectorize=True).numpy()
    return float(np.abs(np.linalg.eigvals(J)).max())


@pytest.mark.parametrize("rho", [1.8, 2.49])
def test_walled_column_stable_at_convection_cell_tc(rho):
    # the convection cell runs at T_c = 0.08 with liquid densities up to 2.49
    assert _walled_column_radius(0.08, rho) < 1 + 1e-9


def test_walled_column_unstable_for_hotter_critical_point():
    # a wall-localised oscillation (about 12 steps per period) grows for the
    # dense liquid once T_c reaches 0.1, which is why the cell stays at 0.08
    assert _walled_column_radius(0.1, 2.49) > 1.002


# ---------------------------------------------------------------- literal readings
# Test-local variants of the step that take the Algorithm section's coupling
# literally, to show why the oracle (and the library) read it differently.

def _variant_step(p, f, g, t_in_feq, explicit_source):
    """One step with (t_in_feq) the dynamic temperature T = E/rho in the
    isotropic second moment of f^eq (through the rest population) and no
    thermal force, and/or (explicit_source) a g equilibrium advecting E with
    v (first moment E v) plus the compressive work -(E/c_v) div v added as
    w_l Q after the collision.  With both False it is the oracle's step."""
    rho, j, E = lbm.hydro_moments(f, g)
    T = E / rho
    grav = torch.stack([torch.zeros_like(rho), torch.zeros_like(rho), -p.gravity * rho])
    if t_in_feq:
        F = lbm.sc_force(p, rho) + grav
        gE = lbm._grad_w(p, E, "linear")
        T_lat = T
    else:
        F, gE, _ = lbm.forces(p, rho, E)
        T_lat = p.T_lattice
    u = (j + p.tau_nu * F) / rho
    v = (j + 0.5 * F) / rho
    feq = lbm.f_equilibrium(rho, u, T_lat)
    w = lbm.W_LAT.view(19, 1, 1, 1)
    if explicit_source:
        cv = torch.einsum("la,azyx->lzyx", lbm.C, v)
        vv = (v * v).sum(0)
        b = lbm.B_G.view(19, 1, 1, 1)
        geq = w * (E + E * (3.0 * cv + 4.5 * cv * cv - 1.5 * vv)) + b * (p.rho_kappa - rho) * T
        Q = -(E / p.c_v) * lbm.divergence(p, v)
    else:
        geq = lbm.g_equilibrium(p, rho, E, v, T)
        Q = (v * gE).sum(0) / p.c_v
    fs = f - (f - feq) / p.tau_nu
    gs = g - (g - geq) / p.tau_kappa + w * Q
    return lbm.stream(p, fs, gs)


def _variant_radii(p, T0, rho0, **kw):
    n = p.nx
    shape = (1, 1, n)
    f, g = lbm.init_state(p, torch.full(shape, rho0, dtype=DT), torch.full(shape, T0, dtype=DT))
    s0 = torch.cat([f, g]).reshape(-1)

    def fn(s):
        s = s.view(38, *shape)
        a, b = _variant_step(p, s[:19], s[19:], **kw)
        return torch.cat([a, b]).reshape(-1)

    J = torch.autograd.functional.jacobian(fn, s0, vectorize=True).numpy().reshape(38, n, 38, n)
    return [np.abs(np.linalg.eigvals(sum(J[:, x, :, 0] * np.exp(-2j * np.pi * m * x / n)
                                          for x in range(n)))).max() for m in range(n // 2 + 1)]


def test_variant_step_with_nothing_literal_is_the_oracle_step():
    p = lbm.Params(6, 1, 5, tau_nu=0.7, tau_kappa=0.8, G=eos.coupling_for_tc(0.05), gravity=1e-4)
    rho0 = torch.tensor(np.random.default_rng(1).uniform(1.6, 2.0, (5, 1, 6)))
    f, g = lbm.init_state(p, rho0)
    a, b = _variant_step(p, f, g, False, False)
    c, d = lbm.step(p, f, g)
    assert torch.equal(a, c) and torch.equal(b, d)


@pytest.mark.parametrize("state", [(0.9, 1.8), (0.97, 2.0)])
def test_literal_temperature_in_feq_is_unstable_at_the_paper_viscosity(state):
    """The dynamic T in f^eq's rest population (the coupling paragraph read
    literally) makes liquid rest states grow at tau_nu = 0.5495 (Table 1's
    nu): spectral radius about 1.07-1.08 per step, where the split reading
    (constant T_lat in f^eq, rho (T - T_lat) as a force) stays on the unit
    circle."""
    Tc = 0.05
    p = lbm.Params(16, 1, 1, tau_nu=0.5495, tau_kappa=0.6417, G=eos.coupling_for_tc(Tc),
                   periodic_z=True)
    lit = _variant_radii(p, state[0] * Tc, state[1], t_in_feq=True, explicit_source=False)
    ours = _variant_radii(p, state[0] * Tc, state[1], t_in_feq=False, explicit_source=False)
    assert max(lit) > 1.05
    assert max(ours) < 1 + 1e-9


@pytest.mark.parametrize("state", [(0.9, 1.8), (1.5, 1.0)])
def test_explicit_counter_term_anti_damps_sound_at_low_viscosity(state):
    """The compressive work added explicitly as -(E/c_v) div v (first order in
    time) lets long sound waves grow at low viscosity (tau = 0.52, ideal
    gas): |lambda| > 1 at the lowest wavenumbers, where the flux form (gamma
    E v in g^eq plus v . grad E / c_v) is stable.  At the paper's tau_nu both
    are stable; the flux form is kept."""
    Tc = 0.05
    p = lbm.Params(32, 1, 1, tau_nu=0.52, tau_kappa=0.52, G=0.0, periodic_z=True,
                   T_lat=state[0] * Tc, T_d=state[0] * Tc, T_u=state[0] * Tc)
    expl = _variant_radii(p, state[0] * Tc, state[1], t_in_feq=False, explicit_source=True)
    ours = _variant_radii(p, state[0] * Tc, state[1], t_in_feq=False, explicit_source=False)
    assert max(expl) > 1 + 1e-4
    assert int(np.argmax(expl)) <= 4          # a long-wave (sound) mode
    assert max(ours) < 1 + 1e-9


def test_stability_limit_in_tau_kappa():
    """The scheme's own stability domain in the conductivity: at tau_nu =
    0.6 an ideal gas at rest (rho 1, T 0.075) is stable for tau_kappa = 1
    and grows at the grid scale for tau_kappa = 2 (radius about 1.009 near
    k = pi).  Every workload here has tau_kappa <= 1 (Table 1's diffusivities
    give tau_kappa ~ 0.6)."""
    for tk, bound in ((1.0, None), (2.0, 1.005)):
        p = lbm.Params(32, 1, 1, tau_nu=0.6, tau_kappa=tk, G=0.0, periodic_z=True,
                       T_lat=0.075, T_d=0.075, T_u=0.075)
        r = _variant_radii(p, 0.075, 1.0, t_in_feq=False, explicit_source=False)
        if bound is None:
            assert max(r) < 1 + 1e-9
        else:
            assert max(r) > bound and int(np.argmax(r)) >= 12
