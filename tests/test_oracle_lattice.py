"""Pins of the oracle's lattice tables and equilibria.

Each check is a property the paper or the textbook D3Q19 lattice fixes, not a
retyping of the oracle's own formula:
* lattice weights: normalisation, zero odd moments, second moment c_s^2 = 1/3,
  fourth-order isotropy (textbook D3Q19);
* force weights: eq. (FORCE) asks for isotropy up to 4th order; with the
  normalisation sum W c c = 1 the bulk pressure becomes (G/2) exp(-2/rho);
* f^eq moments: rho, rho u', rho T_lat delta + rho u'u' (polynomial
  equilibrium of the lattice with the lattice temperature T_lat);
* g^eq moments: rho T, gamma rho T v_g, and an isotropic second moment
  independent of the local density (one conductivity in both phases,
  Table 1);
* the thermal force reproduces the ideal pressure gradient: for G = 0 the
  net force F - grad(rho T_lat) (lattice pressure) equals -grad(rho T).
"""
import itertools

import pytest
import torch

from oracle import lbm

C = lbm.C
W = lbm.W_LAT
WF = lbm.W_FOR


def _moment(w, idx):
    out = w.clone()
    for a in idx:
        out = out * C[:, a]
    return out.sum().item()


def _iso4(a, b, c, d):
    k = lambda i, j: 1.0 if i == j else 0.0  # noqa: E731
    return k(a, b) * k(c, d) + k(a, c) * k(b, d) + k(a, d) * k(b, c)


def test_velocity_set_shape():
    vecs = [tuple(int(x) for x in row) for row in C.tolist()]
    assert len(set(vecs)) == 19
    norms = sorted(sum(x * x for x in v) for v in vecs)
    assert norms == [0] + [1] * 6 + [2] * 12
    for l, o in enumerate(lbm.OPP):
        assert all(a == -b for a, b in zip(vecs[l], vecs[o]))


def test_lattice_weight_moments():
    assert abs(W.sum().item() - 1.0) < 1e-15
    for a in range(3):
        assert abs(_moment(W, [a])) < 1e-15
    for a, b in itertools.product(range(3), repeat=2):
        assert abs(_moment(W, [a, b]) - (1 / 3 if a == b else 0)) < 1e-15
        for c in range(3):
            assert abs(_moment(W, [a, b, c])) < 1e-15
    for idx in itertools.product(range(3), repeat=4):
        assert abs(_moment(W, list(idx)) - _iso4(*idx) / 9.0) < 1e-15


def test_force_weights_isotropic_to_fourth_order():
    for a, b in itertools.product(range(3), repeat=2):
        assert abs(_moment(WF, [a, b]) - (1.0 if a == b else 0.0)) < 1e-15
    m4 = {idx: _moment(WF, list(idx)) for idx in itertools.product(range(3), repeat=4)}
    lam = m4[(0, 0, 1, 1)]
    for idx, val in m4.items():
        assert abs(val - lam * _iso4(*idx)) < 1e-15
    assert lam > 0


def _random_fields(n=5, seed=0):
    gen = torch.Generator().manual_seed(seed)
    rho = 0.5 + 1.5 * torch.rand((1, 1, n), generator=gen, dtype=torch.float64)
    u = 0.1 * (torch.rand((3, 1, 1, n), generator=gen, dtype=torch.float64) - 0.5)
    T = 0.2 + 0.3 * torch.rand((1, 1, n), generator=gen, dtype=torch.float64)
    return rho, u, T


@pytest.mark.parametrize("T_lat", [1.0 / 3.0, 0.045])
def test_f_equilibrium_moments(T_lat):
    rho, u, T = _random_fields()
    feq = lbm.f_equilibrium(rho, u, T_lat)
    assert torch.allclose(feq.sum(0), rho, rtol=0, atol=1e-14)
    j = torch.einsum("la,lzyx->azyx", C, feq)
    assert torch.allclose(j, rho * u, rtol=0, atol=1e-14)
    for a, b in itertools.product(range(3), repeat=2):
        m2 = (C[:, a].view(19, 1, 1, 1) * C[:, b].view(19, 1, 1, 1) * feq).sum(0)
        want = rho * u[a] * u[b] + (rho * T_lat if a == b else 0.0)
        assert torch.allclose(m2, want, rtol=0, atol=1e-14)


def test_g_equilibrium_moments():
    rho, v, T = _random_fields(seed=1)
    vl = v + 0.01
    p = lbm.Params(1, 1, 5, rho_kappa=0.7, c_v=1.5)
    gam = 1 + 1 / p.c_v
    E = rho * T
    geq = lbm.g_equilibrium(p, rho, E, v, T, v_lin=vl)
    assert torch.allclose(geq.sum(0), E, rtol=0, atol=1e-14)
    flux = torch.einsum("la,lzyx->azyx", C, geq)
    assert torch.allclose(flux, gam * E * vl, rtol=0, atol=1e-14)
    for a, b in itertools.product(range(3), repeat=2):
        m2 = (C[:, a].view(19, 1, 1, 1) * C[:, b].view(19, 1, 1, 1) * geq).sum(0)
        want = gam * E * v[a] * v[b] + (p.rho_kappa * T / 3.0 if a == b else 0.0)
        assert torch.allclose(m2, want, rtol=0, atol=1e-14)


def test_thermal_force_gives_ideal_pressure_gradient():
    """G = 0, no gravity: F - (lattice pressure gradient of rho T_lat) is the
    W-stencil gradient of -rho T, i.e. the fluid feels P0 = rho T."""
    n = 64
    p = lbm.Params(1, 1, n, G=0.0, periodic_z=True)
    z = torch.arange(n, dtype=torch.float64)
    k = 2 * torch.pi / n
    rho = (1.0 + 0.2 * torch.sin(k * z)).view(n, 1, 1)
    T = (0.09 + 0.01 * torch.cos(k * z)).view(n, 1, 1)
    F, gE, grho = lbm.forces(p, rho, rho * T)
    P0 = (rho * T).view(n)
    dP = (torch.roll(P0, -1) - torch.roll(P0, 1)) / 2   # central difference
    got = F[2].view(n) - p.T_lattice * grho[2].view(n)   # force minus lattice pressure gradient
    assert torch.allclose(got, -dP, rtol=0, atol=1e-15)


def test_pseudopotential_and_force_match_eos_gradient():
    """A smooth density field: F_SC -> -(G/2) grad exp(-2/rho) (bulk P_NI)."""
    n = 256
    p = lbm.Params(1, 1, n, G=-2.5, periodic_z=True)
    z = torch.arange(n, dtype=torch.float64)
    k = 2 * torch.pi / n
    rho = (1.2 + 0.3 * torch.sin(k * z)).view(n, 1, 1)
    F = lbm.sc_force(p, rho)
    drho = 0.3 * k * torch.cos(k * z)
    want = -(p.G / 2.0) * torch.exp(-2.0 / rho.view(n)) * (2.0 / rho.view(n) ** 2) * drho
    err = (F[2].view(n) - want).abs().max() / want.abs().max()
    assert err < 2e-3  # second-order stencil at k = 2 pi / 256
    assert F[0].abs().max() < 1e-15 and F[1].abs().max() < 1e-15
