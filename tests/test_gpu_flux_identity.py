"""eq. (flux) on a steady convecting state.

Integrating the layer heat balance eq. (heat2) over time at a statistically
steady state leaves d/dz <rho U v_z - kappa dT/dz> = -<P d_j v_j>: the heat
flux changes across the layer only by the plane-averaged pressure work, so
Nu(z) - Nu(0) is minus its integral (eq. (flux)).  A strongly stratified
ideal gas (G = 0, T_m = 0.05, beta dT = 0.3, the adiabatic gradient 21 % of
the imposed one) in a 64 x 1 x 32 cell at 3.3 Ra_c settles into a steady roll
within 4e4 steps; there Nu(z) runs from about 1.06 to 1.96, and the central
difference of the flux profile (lbm_nusselt) must match minus the pressure
work profile (lbm_pressure_work) to the truncation error of the differences,
while dropping the work term misses by the size of the terms.

This is a property of the discrete model at any size, checked through the
library on the FP64 path (which equals the oracle step to 1e-12, per the
parity tests) and on FP32 storage; the oracle cannot reach the steady state in
test time.
"""
import math

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

H, NX = 32, 64
T_M, C_V, RHO_K = 0.05, 1.0, 0.5
C_P = C_V + 1.0
BETA = 1.0 / T_M
DT = 0.3 / BETA
TAU = 0.55
NU = (TAU - 0.5) / 3.0
CHI = NU
G_GRAV = 2e-4


@pytest.fixture(scope="module")
def glbm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1111_0905_amd import lbm
    lbm.load_library()
    return lbm


def _cell(glbm, storage):
    kappa = CHI * 1.0 * C_P
    p = glbm.Params(NX, 1, H, storage=storage, tau_nu=TAU, tau_kappa=0.5 + 3 * kappa / (C_V * RHO_K),
                    G=0.0, T_d=T_M + DT / 2, T_u=T_M - DT / 2, gravity=G_GRAV, c_v=C_V,
                    rho_kappa=RHO_K, T_lat=T_M, rho_ref=1.0, T_ref=T_M)
    z = np.arange(H) + 0.5
    Tz = p.T_d + (p.T_u - p.T_d) * z / H
    # hydrostatic ideal gas on the nodes: P = rho T, P_{k+1} - P_k = -g (rho_k + rho_{k+1}) / 2
    rho = [1.0]
    for k in range(1, H):
        rho.append(rho[-1] * (Tz[k - 1] - G_GRAV / 2) / (Tz[k] + G_GRAV / 2))
    rho = np.array(rho) / np.mean(rho)
    x = np.arange(NX) + 0.5
    T0 = Tz[:, None] + 3e-2 * DT * np.sin(math.pi * z / H)[:, None] * np.sin(2 * math.pi * x / NX)[None, :]
    rho0 = np.repeat(rho[:, None], NX, axis=1)
    lat = glbm.Lattice(p, torch.from_numpy(rho0.ravel().copy()).cuda(),
                       torch.from_numpy(T0.ravel().copy()).cuda())
    return lat, kappa * DT / H


@pytest.mark.parametrize("storage", ["fp64", "fp32"])
def test_flux_constraint_on_a_steady_roll(glbm, storage):
    st = {"fp64": glbm.LBM_FP64, "fp32": glbm.LBM_FP32}[storage]
    print(f"case: steady roll {NX}x1x{H}, {storage}", flush=True)
    lat, qref = _cell(glbm, st)
    lat.step(40000)
    _, _, nu_a, _ = lat.nusselt()
    lat.step(2000)
    nb, nt, nu_z, _ = lat.nusselt()
    pw = lat.pressure_work()
    # steady: the profile no longer moves
    assert np.abs(nu_z - nu_a).max() < 1e-4 * np.abs(nu_z).max()
    F = np.asarray(nu_z) * qref
    div = 0.5 * (F[2:] - F[:-2])
    res = div + pw[1:-1]
    scale = np.abs(pw).max()
    print(f"{storage}: Nu_bot {nb:.4f} Nu_top {nt:.4f}, Nu(z) in [{nu_z.min():.3f}, {nu_z.max():.3f}]; "
          f"max|dF/dz| {np.abs(div).max():.3e}, max|PW| {scale:.3e}, "
          f"max|dF/dz + PW| {np.abs(res).max():.3e} ({np.abs(res).max() / scale:.3f} of the terms)")
    # a convecting state whose flux changes across the layer by the pressure work
    assert nu_z.max() - nu_z.min() > 0.5
    assert np.abs(res).max() < 0.1 * scale
    # without the work term the balance misses by the size of the terms
    assert np.abs(div).max() > 0.8 * scale
