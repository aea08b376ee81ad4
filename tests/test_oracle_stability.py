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
