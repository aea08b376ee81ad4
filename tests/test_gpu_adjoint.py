"""GPU adjoint against the oracle's own discrete adjoint (autograd of the
torch-CPU FP64 oracle) and against central finite differences.

Bars (FP64 handles): one adjoint step 1e-11 relative; trajectory gradients
dJ/dT_d, dJ/dG and dJ/drho0 1e-9 relative to the oracle's; central finite
differences (h = 1e-4 relative for T_d and G, 1e-6 along a seeded direction
for rho0) within 1e-4 relative.
"""
import math

import numpy as np
import pytest
import torch

import synth
from oracle import eos
from oracle import lbm as olbm

pytestmark = pytest.mark.gpu

TC = 0.05
G = eos.coupling_for_tc(TC)


@pytest.fixture(scope="module")
def glbm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1111_0905_amd import lbm
    lbm.load_library()
    return lbm


def _kw(**over):
    kw = dict(tau_nu=0.8, tau_kappa=0.7, G=G, T_d=0.95 * TC, T_u=0.85 * TC, gravity=1e-4)
    kw.update(over)
    return kw


def _rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("storage", ["fp64", "fp32"])
@pytest.mark.parametrize("periodic", [0, 1])
@pytest.mark.parametrize("shape", [(6, 5, 7), (9, 4, 2)])
def test_one_step_adjoint_matches_oracle_vjp(glbm, periodic, shape, storage):
    # the adjoint arithmetic is FP64 for every storage form, so an FP32 handle
    # linearises about the given FP64 state exactly as an FP64 handle does
    nx, ny, nz = shape
    print(f"case: one-step adjoint {shape} periodic={periodic} {storage}", flush=True)
    kw = _kw()
    p_o = olbm.Params(nx, ny, nz, periodic_z=bool(periodic), **kw)
    rho0 = synth.noisy_density(nx, ny, nz, 1.9, 0.05, 21)
    f, g = olbm.init_state(p_o, torch.from_numpy(rho0))
    for _ in range(3):
        f, g = olbm.step(p_o, f, g)
    s = torch.cat([f, g]).detach()
    lam = torch.from_numpy(np.random.default_rng(5).standard_normal(s.shape))
    # oracle VJP, with the parameters as leaves
    s_r = s.clone().requires_grad_(True)
    Gt = torch.tensor(kw["G"], dtype=torch.float64, requires_grad=True)
    Tdt = torch.tensor(kw["T_d"], dtype=torch.float64, requires_grad=True)
    fo, go = olbm.step(p_o, s_r[:19], s_r[19:], G=Gt, T_d=Tdt)
    out = torch.cat([fo, go])
    ds, dG, dTd = torch.autograd.grad(out, [s_r, Gt, Tdt], grad_outputs=lam, allow_unused=True)
    # GPU adjoint
    p_g = glbm.Params(nx, ny, nz, storage=glbm.STORAGE[storage], periodic_z=periodic, adjoint=1,
                      **kw)
    lat = glbm.Lattice(p_g, torch.from_numpy(rho0).cuda())
    st = s.cuda().contiguous()
    lam_g = lam.cuda().contiguous()
    out_g = torch.empty_like(lam_g)
    grads = np.zeros(2)
    glbm.lbm_adjoint_step(lat.h, st, lam_g, out_g, grads)
    assert _rel(out_g.cpu().numpy(), ds.numpy()) < 1e-11
    assert abs(grads[0] - dG.item()) < 1e-11 * max(1.0, abs(dG.item()))
    want_Td = 0.0 if (periodic or dTd is None) else dTd.item()
    assert abs(grads[1] - want_Td) < 1e-11 * max(1.0, abs(want_Td))


def test_one_step_adjoint_with_wetting_walls(glbm):
    # a prescribed wall density makes the psi ghost a constant: its adjoint
    # drops out of the stencil transpose
    nx, ny, nz = 6, 5, 7
    print("case: one-step adjoint with wetting walls", flush=True)
    kw = _kw(rho_wall_d=2.2, rho_wall_u=0.7)
    p_o = olbm.Params(nx, ny, nz, **kw)
    rho0 = synth.noisy_density(nx, ny, nz, 1.9, 0.05, 23)
    f, g = olbm.init_state(p_o, torch.from_numpy(rho0))
    for _ in range(3):
        f, g = olbm.step(p_o, f, g)
    s = torch.cat([f, g]).detach()
    lam = torch.from_numpy(np.random.default_rng(6).standard_normal(s.shape))
    s_r = s.clone().requires_grad_(True)
    Gt = torch.tensor(kw["G"], dtype=torch.float64, requires_grad=True)
    Tdt = torch.tensor(kw["T_d"], dtype=torch.float64, requires_grad=True)
    fo, go = olbm.step(p_o, s_r[:19], s_r[19:], G=Gt, T_d=Tdt)
    ds, dG, dTd = torch.autograd.grad(torch.cat([fo, go]), [s_r, Gt, Tdt], grad_outputs=lam)
    p_g = glbm.Params(nx, ny, nz, storage=glbm.LBM_FP64, adjoint=1, **kw)
    lat = glbm.Lattice(p_g, torch.from_numpy(rho0).cuda())
    lam_g = lam.cuda().contiguous()
    out_g = torch.empty_like(lam_g)
    grads = np.zeros(2)
    glbm.lbm_adjoint_step(lat.h, s.cuda().contiguous(), lam_g, out_g, grads)
    assert _rel(out_g.cpu().numpy(), ds.numpy()) < 1e-11
    assert abs(grads[0] - dG.item()) < 1e-11 * max(1.0, abs(dG.item()))
    assert abs(grads[1] - dTd.item()) < 1e-11 * max(1.0, abs(dTd.item()))


def test_one_step_adjoint_with_sc_pseudopotential(glbm):
    # psi = 1 - exp(-rho): d psi / d rho = exp(-rho) in the local and the
    # stencil parts of the adjoint
    nx, ny, nz = 6, 5, 7
    print("case: one-step adjoint, Shan-Chen psi", flush=True)
    kw = _kw(G=-4 * TC, psi_form=1, rho_wall_u=0.4)
    p_o = olbm.Params(nx, ny, nz, **kw)
    rho0 = synth.noisy_density(nx, ny, nz, 1.0, 0.05, 29)
    f, g = olbm.init_state(p_o, torch.from_numpy(rho0))
    for _ in range(3):
        f, g = olbm.step(p_o, f, g)
    s = torch.cat([f, g]).detach()
    lam = torch.from_numpy(np.random.default_rng(8).standard_normal(s.shape))
    s_r = s.clone().requires_grad_(True)
    Gt = torch.tensor(kw["G"], dtype=torch.float64, requires_grad=True)
    Tdt = torch.tensor(kw["T_d"], dtype=torch.float64, requires_grad=True)
    fo, go = olbm.step(p_o, s_r[:19], s_r[19:], G=Gt, T_d=Tdt)
    ds, dG, dTd = torch.autograd.grad(torch.cat([fo, go]), [s_r, Gt, Tdt], grad_outputs=lam)
    p_g = glbm.Params(nx, ny, nz, storage=glbm.LBM_FP64, adjoint=1, **kw)
    lat = glbm.Lattice(p_g, torch.from_numpy(rho0).cuda())
    lam_g = lam.cuda().contiguous()
    out_g = torch.empty_like(lam_g)
    grads = np.zeros(2)
    glbm.lbm_adjoint_step(lat.h, s.cuda().contiguous(), lam_g, out_g, grads)
    assert _rel(out_g.cpu().numpy(), ds.numpy()) < 1e-11
    assert abs(grads[0] - dG.item()) < 1e-11 * max(1.0, abs(dG.item()))
    assert abs(grads[1] - dTd.item()) < 1e-11 * max(1.0, abs(dTd.item()))


def test_qbot_and_its_adjoint(glbm):
    nx, ny, nz = 7, 6, 5
    kw = _kw()
    p_o = olbm.Params(nx, ny, nz, **kw)
    rho0 = synth.noisy_density(nx, ny, nz, 1.9, 0.05, 2)
    f, g = olbm.init_state(p_o, torch.from_numpy(rho0))
    f, g = olbm.step(p_o, f, g)
    s = torch.cat([f, g]).detach().requires_grad_(True)
    Tdt = torch.tensor(kw["T_d"], dtype=torch.float64, requires_grad=True)
    q = olbm.q_bottom(p_o, s[:19], s[19:], T_d=Tdt)
    ds, dTd = torch.autograd.grad(q, [s, Tdt])
    p_g = glbm.Params(nx, ny, nz, storage=glbm.LBM_FP64, adjoint=1, **kw)
    lat = glbm.Lattice(p_g, torch.from_numpy(rho0).cuda())
    adj = torch.zeros(38 * nx * ny * nz, dtype=torch.float64, device="cuda")
    grads = np.zeros(2)
    qg = glbm.lbm_adjoint_qbot(lat.h, s.detach().cuda().contiguous(), 1.0, adj, grads)
    assert abs(qg - q.item()) < 1e-14
    assert _rel(adj.cpu().numpy().reshape(ds.shape), ds.numpy()) < 1e-12
    assert abs(grads[1] - dTd.item()) < 1e-14


def _oracle_objective_grads(p_o, rho0, n_steps):
    rho = torch.from_numpy(rho0).clone().requires_grad_(True)
    Gt = torch.tensor(p_o.G, dtype=torch.float64, requires_grad=True)
    Tdt = torch.tensor(p_o.T_d, dtype=torch.float64, requires_grad=True)
    T0 = olbm.initial_temperature(p_o)          # fixed initial profile
    f, g = olbm.init_state(p_o, rho, T0)
    J = 0.0
    for _ in range(n_steps):
        f, g = olbm.step(p_o, f, g, G=Gt, T_d=Tdt)
        J = J + olbm.q_bottom(p_o, f, g, T_d=Tdt)
    J = J / n_steps
    dr, dG, dTd = torch.autograd.grad(J, [rho, Gt, Tdt])
    return J.item(), dr.numpy(), dG.item(), dTd.item()


def test_trajectory_gradients_match_oracle_adjoint(glbm):
    from paper_1111_0905_amd import adjoint
    n = 16
    n_steps = 12
    print("case: 16^3 trajectory gradients, 12 steps, checkpoint every 5", flush=True)
    kw = _kw(tau_nu=1.0, tau_kappa=1.0, gravity=1e-5)
    rg, rl, _ = eos.maxwell(0.9 * TC, G)
    rho0 = synth.noisy_density(n, n, n, 0.5 * (rg + rl), 0.01, 1234)
    J_o, dr_o, dG_o, dTd_o = _oracle_objective_grads(olbm.Params(n, n, n, **kw), rho0, n_steps)
    p = glbm.Params(n, n, n, storage=glbm.LBM_FP64, **kw)
    J, dr, dTd, dG = adjoint.heat_flux_gradients(p, torch.from_numpy(rho0), n_steps, ckpt_every=5)
    assert abs(J - J_o) < 1e-12 * abs(J_o)
    assert abs(dTd / dTd_o - 1) < 1e-9
    assert abs(dG / dG_o - 1) < 1e-9
    assert _rel(dr.cpu().numpy().reshape(dr_o.shape), dr_o) < 1e-9


def test_gradients_match_central_differences(glbm):
    from paper_1111_0905_amd import adjoint
    n = 12
    n_steps = 10
    print("case: 12^3 FD check, 10 steps", flush=True)
    # T_lat held at its value for the unperturbed T_d (the gradient's convention)
    kw = _kw(tau_nu=1.0, tau_kappa=1.0, gravity=1e-5, T_lat=0.9 * TC)
    rho0 = torch.from_numpy(synth.noisy_density(n, n, n, 1.18, 0.01, 99)).cuda().reshape(-1)
    p = glbm.Params(n, n, n, storage=glbm.LBM_FP64, **kw)
    T0 = adjoint.conduction_profile(p)
    J, dr, dTd, dG = adjoint.heat_flux_gradients(p, rho0, n_steps, ckpt_every=4, T0=T0)

    from dataclasses import replace
    h = 1e-4 * p.T_d
    fd_Td = (adjoint.heat_flux_objective(replace(p, T_d=p.T_d + h), rho0, n_steps, T0) -
             adjoint.heat_flux_objective(replace(p, T_d=p.T_d - h), rho0, n_steps, T0)) / (2 * h)
    h = 1e-4 * abs(p.G)
    fd_G = (adjoint.heat_flux_objective(replace(p, G=p.G + h), rho0, n_steps, T0) -
            adjoint.heat_flux_objective(replace(p, G=p.G - h), rho0, n_steps, T0)) / (2 * h)
    d = torch.from_numpy(synth.random_unit_field(n, n, n, 7)).cuda().reshape(-1)
    h = 1e-6
    fd_r = (adjoint.heat_flux_objective(p, rho0 + h * d, n_steps, T0) -
            adjoint.heat_flux_objective(p, rho0 - h * d, n_steps, T0)) / (2 * h)
    ad_r = float((dr * d).sum())
    print(f"FD vs adjoint: T_d {fd_Td:.8e} {dTd:.8e}; G {fd_G:.8e} {dG:.8e}; rho0 {fd_r:.8e} {ad_r:.8e}")
    assert abs(fd_Td / dTd - 1) < 1e-4
    assert abs(fd_G / dG - 1) < 1e-4
    assert abs(fd_r / ad_r - 1) < 1e-4


def test_autograd_function(glbm):
    from paper_1111_0905_amd import adjoint
    n = 8
    kw = _kw(tau_nu=1.0, tau_kappa=1.0, gravity=1e-5)
    p = glbm.Params(n, n, n, storage=glbm.LBM_FP64, **kw)
    rho0 = torch.from_numpy(synth.noisy_density(n, n, n, 1.18, 0.01, 3)).cuda().reshape(-1)
    rho0.requires_grad_(True)
    Td = torch.tensor(p.T_d, dtype=torch.float64, requires_grad=True)
    Gt = torch.tensor(p.G, dtype=torch.float64, requires_grad=True)
    J = adjoint.HeatFluxObjective.apply(rho0, Td, Gt, p, 6, 3)
    J.backward()
    J2, dr, dTd, dG = adjoint.heat_flux_gradients(p, rho0.detach(), 6, 3)
    assert abs(J.item() - J2) < 1e-15
    assert torch.equal(rho0.grad, dr)
    assert Td.grad.item() == dTd and Gt.grad.item() == dG


def test_autograd_function_matches_its_own_finite_differences(glbm):
    """HeatFluxObjective differentiated against central differences of its
    own forward in T_d (h = 1e-4 relative), FP64, 8^3, T_lat left at its
    default: the forward pins T_lat (and T0) at the values of the given
    parameters, so the derivative the adjoint returns is that of the
    function's own output."""
    from paper_1111_0905_amd import adjoint
    n = 8
    kw = _kw(tau_nu=1.0, tau_kappa=1.0, gravity=1e-5)
    p = glbm.Params(n, n, n, storage=glbm.LBM_FP64, **kw)
    assert p.T_lat == 0.0
    rho0 = torch.from_numpy(synth.noisy_density(n, n, n, 1.18, 0.01, 3)).cuda().reshape(-1)
    Gt = torch.tensor(p.G, dtype=torch.float64)
    Td = torch.tensor(p.T_d, dtype=torch.float64, requires_grad=True)
    J = adjoint.HeatFluxObjective.apply(rho0, Td, Gt, p, 6, 3)
    J.backward()
    h = 1e-4 * p.T_d
    Jp = adjoint.HeatFluxObjective.apply(rho0, torch.tensor(p.T_d + h, dtype=torch.float64), Gt, p, 6, 3)
    Jm = adjoint.HeatFluxObjective.apply(rho0, torch.tensor(p.T_d - h, dtype=torch.float64), Gt, p, 6, 3)
    fd = (Jp.item() - Jm.item()) / (2 * h)
    print(f"dJ/dT_d adjoint {Td.grad.item():.10e} central difference {fd:.10e}")
    assert abs(Td.grad.item() - fd) < 1e-4 * abs(fd)
