"""Domain of dependence of the step, which the full-size sampled parity test
relies on: the state of a node after s steps depends only on the initial
state within 2 s nodes of it in x and y (forces at a neighbour use psi, rho
and E one node further out; streaming moves one node), so a periodic patch of
width 4 s + 1 cut around a column reproduces that column exactly, and a patch
of width 4 s - 1 does not."""
import numpy as np
import torch

import synth
from oracle import eos, lbm

TC = 0.05
G = eos.coupling_for_tc(TC)


def _run(nx, ny, nz, rho0, steps):
    p = lbm.Params(nx, ny, nz, tau_nu=0.7, tau_kappa=0.8, G=G, T_d=0.95 * TC, T_u=0.85 * TC,
                   gravity=1e-4)
    o = lbm.Oracle(p, np.ascontiguousarray(rho0))
    o.step(steps)
    return o.state().numpy()


def _patch(rho0, x, y, half):
    ny, nx = rho0.shape[1:]
    xs = [(x + d) % nx for d in range(-half, half + 1)]
    ys = [(y + d) % ny for d in range(-half, half + 1)]
    return rho0[:, ys][:, :, xs]


def test_patch_of_width_4s_plus_1_reproduces_the_centre_column():
    steps = 3
    nx, ny, nz = 26, 23, 7
    rho0 = synth.noisy_density(nx, ny, nz, 1.9, 0.08, 17)
    full = _run(nx, ny, nz, rho0, steps)
    for (x, y) in [(0, 0), (25, 11), (13, 22)]:
        h = 2 * steps
        sub = _run(2 * h + 1, 2 * h + 1, nz, _patch(rho0, x, y, h), steps)
        assert np.abs(sub[:, :, h, h] - full[:, :, y, x]).max() < 1e-13
        # one node less on each side is not enough
        h2 = 2 * steps - 1
        sub2 = _run(2 * h2 + 1, 2 * h2 + 1, nz, _patch(rho0, x, y, h2), steps)
        assert np.abs(sub2[:, :, h2, h2] - full[:, :, y, x]).max() > 1e-10
