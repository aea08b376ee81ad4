"""Exact discrete invariants of the oracle step (no tolerance beyond roundoff).

* mass: streaming, bounce-back and BGK collision conserve sum f;
* momentum: the pair force of eq. (FORCE) is antisymmetric, so on a fully
  periodic lattice sum j changes per step by exactly the total body force
  -M g z-hat (the velocity shift puts exactly F into the collided moments);
* rest state: uniform rho and T at rest is a fixed point, with and without
  walls (neutral ghost density at the walls);
* lattice symmetries: integer shifts in x, y, the x<->y swap, and the
  reflection z -> nz-1-z together with T_d <-> T_u and g -> -g commute with
  the step.
"""
import math

import torch

import synth
from oracle import lbm

TC = 0.05
G = -TC * math.e ** 2


def _state(p, mean=2.6, amp=0.05, seed=7):
    rho0 = torch.from_numpy(synth.noisy_density(p.nx, p.ny, p.nz, mean, amp, seed))
    f, g = lbm.init_state(p, rho0)
    # a few steps so that velocities and the counter-term are non-trivial
    for _ in range(3):
        f, g = lbm.step(p, f, g)
    return f, g


def test_mass_conserved_with_walls():
    p = lbm.Params(6, 5, 7, tau_nu=0.8, tau_kappa=0.7, G=G, T_d=0.048, T_u=0.042, gravity=1e-3)
    f, g = _state(p)
    m0 = f.sum().item()
    for _ in range(20):
        f, g = lbm.step(p, f, g)
    assert abs(f.sum().item() - m0) / m0 < 1e-14


def test_momentum_conserved_periodic():
    p = lbm.Params(6, 5, 7, tau_nu=0.8, tau_kappa=0.7, G=G, gravity=0.0, periodic_z=True)
    f, g = _state(p, amp=0.08)
    j0 = torch.einsum("la,lzyx->a", lbm.C, f)
    scale = torch.einsum("la,lzyx->azyx", lbm.C, f).abs().sum().item()
    for _ in range(10):
        f, g = lbm.step(p, f, g)
    j1 = torch.einsum("la,lzyx->a", lbm.C, f)
    assert (j1 - j0).abs().max().item() < 1e-13 * max(scale, 1.0)


def test_momentum_gains_exactly_gravity():
    grav = 1e-3
    p = lbm.Params(6, 5, 7, tau_nu=0.8, tau_kappa=0.7, G=G, gravity=grav, periodic_z=True)
    f, g = _state(p, amp=0.08)
    M = f.sum().item()
    for _ in range(5):
        j0 = torch.einsum("la,lzyx->a", lbm.C, f)
        f, g = lbm.step(p, f, g)
        j1 = torch.einsum("la,lzyx->a", lbm.C, f)
        d = (j1 - j0)
        assert abs(d[0].item()) < 1e-12 and abs(d[1].item()) < 1e-12
        assert abs(d[2].item() + M * grav) < 1e-12 * M


def _uniform(p, rho=1.3, T=0.045):
    shape = (p.nz, p.ny, p.nx)
    return lbm.init_state(p, torch.full(shape, rho, dtype=torch.float64),
                          torch.full(shape, T, dtype=torch.float64))


def test_rest_state_is_fixed_point_periodic():
    p = lbm.Params(4, 3, 5, tau_nu=0.7, tau_kappa=0.9, G=G, periodic_z=True)
    f, g = _uniform(p)
    f1, g1 = lbm.step(p, f, g)
    assert (f1 - f).abs().max() < 1e-14 and (g1 - g).abs().max() < 1e-14


def test_rest_state_is_fixed_point_with_walls():
    p = lbm.Params(4, 3, 5, tau_nu=0.7, tau_kappa=0.9, G=G, T_d=0.045, T_u=0.045)
    f, g = _uniform(p)
    f1, g1 = lbm.step(p, f, g)
    assert (f1 - f).abs().max() < 1e-14 and (g1 - g).abs().max() < 1e-14


def _perm(transform):
    vecs = [tuple(v) for v in lbm.C_INT]
    return [vecs.index(transform(v)) for v in vecs]


def test_shift_invariance():
    p = lbm.Params(6, 5, 7, tau_nu=0.8, tau_kappa=0.7, G=G, T_d=0.048, T_u=0.042, gravity=1e-3)
    f, g = _state(p)
    a = lbm.step(p, f, g)
    b = lbm.step(p, torch.roll(f, (2, 3), (2, 3)), torch.roll(g, (2, 3), (2, 3)))
    # equal up to the summation order of the library's reductions
    assert (torch.roll(a[0], (2, 3), (2, 3)) - b[0]).abs().max() < 1e-14
    assert (torch.roll(a[1], (2, 3), (2, 3)) - b[1]).abs().max() < 1e-14


def test_xy_swap_symmetry():
    p = lbm.Params(5, 5, 6, tau_nu=0.8, tau_kappa=0.7, G=G, T_d=0.048, T_u=0.042, gravity=1e-3)
    f, g = _state(p)
    perm = _perm(lambda v: (v[1], v[0], v[2]))

    def swap(x):
        return x[perm].transpose(2, 3)

    a = lbm.step(p, f, g)
    b = lbm.step(p, swap(f), swap(g))
    assert (swap(a[0]) - b[0]).abs().max() < 1e-14
    assert (swap(a[1]) - b[1]).abs().max() < 1e-14


def test_z_reflection_symmetry():
    p = lbm.Params(4, 5, 6, tau_nu=0.8, tau_kappa=0.7, G=G, T_d=0.048, T_u=0.042, gravity=1e-3)
    q = p.with_(T_d=p.T_u, T_u=p.T_d, gravity=-p.gravity)
    f, g = _state(p)
    perm = _perm(lambda v: (v[0], v[1], -v[2]))

    def refl(x):
        return torch.flip(x[perm], dims=(1,))

    a = lbm.step(p, f, g)
    b = lbm.step(q, refl(f), refl(g))
    assert (refl(a[0]) - b[0]).abs().max() < 1e-14
    assert (refl(a[1]) - b[1]).abs().max() < 1e-14
