"""Rayleigh-Benard onset with no-slip walls (the conductive state loses
stability near Ra = 1708; text around eq. (heat2) and Table 1's Ra with the
adiabatic correction), on the FP64 GPU path, which equals the oracle to 1e-12
per step (test_gpu_parity): the growth times near onset (~10^5 steps on a
64-node-high cell) are beyond the CPU oracle's reach.

Weakly stratified ideal gas (G = 0): T_m = 0.05, beta = 1/T, c_p = 2,
beta dT = 0.1, Pr = 1, tau_nu = 0.55; cell 128 x 1 x 64 (k H = pi, next to the
critical k_c H = 3.117); hydrostatic initial density, a 1e-3 dT temperature
mode sin(k x) sin(pi z / H).  The growth rate of the k-mode of v_z at mid
height is negative at 0.8 Ra_c and positive at 1.25 Ra_c, Ra = g beta H^4
(dT/H - gamma_ad) / (chi nu), gamma_ad = beta T g / c_p.
"""
import math

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

H, NX = 64, 128
T_M, C_V = 0.05, 1.0
C_P = C_V + 1.0               # ideal gas: c_p - c_v = T / (dP/drho)_T = 1
BETA = 1.0 / T_M
DT = 0.1 / BETA
TAU_NU = 0.55
NU = (TAU_NU - 0.5) / 3.0
CHI = NU                      # Pr = 1
RHO_K = 0.5


@pytest.fixture(scope="module")
def glbm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1111_0905_amd import lbm
    lbm.load_library()
    return lbm


def _gravity(Ra):
    a = BETA * BETA * T_M * H ** 4 / C_P
    b = -BETA * H ** 3 * DT
    c = Ra * CHI * NU
    return (-b - math.sqrt(b * b - 4 * a * c)) / (2 * a)


def _growth(glbm, Ra, steps=150000, every=5000):
    g = _gravity(Ra)
    kappa = CHI * 1.0 * C_P
    p = glbm.Params(NX, 1, H, storage=glbm.LBM_FP64, tau_nu=TAU_NU,
                    tau_kappa=0.5 + 3 * kappa / (C_V * RHO_K), G=0.0, T_d=T_M + DT / 2,
                    T_u=T_M - DT / 2, gravity=g, c_v=C_V, rho_kappa=RHO_K, T_lat=T_M)
    z = np.arange(H) + 0.5
    Tz = p.T_d + (p.T_u - p.T_d) * z / H
    # hydrostatic ideal gas on the nodes: P = rho T, P_{k+1} - P_k = -g (rho_k + rho_{k+1}) / 2
    rho = [1.0]
    for k in range(1, H):
        rho.append(rho[-1] * (Tz[k - 1] - g / 2) / (Tz[k] + g / 2))
    rho = np.array(rho) / np.mean(rho)
    x = np.arange(NX) + 0.5
    T0 = Tz[:, None] + 1e-3 * DT * np.sin(math.pi * z / H)[:, None] * np.sin(2 * math.pi * x / NX)[None, :]
    rho0 = np.repeat(rho[:, None], NX, axis=1)
    lat = glbm.Lattice(p, torch.from_numpy(rho0.ravel().copy()).cuda(),
                       torch.from_numpy(T0.ravel().copy()).cuda())
    amps = []
    for s in range(every, steps + 1, every):
        lat.step(every)
        _, fl = lat.fields()
        vz = fl[3, H // 2, 0].cpu().numpy()
        amps.append((s, abs(np.fft.rfft(vz)[1])))
    t = np.array([a[0] for a in amps], dtype=float)
    la = np.log(np.array([a[1] for a in amps]))
    half = len(t) // 2
    return float(np.polyfit(t[half:], la[half:], 1)[0])


def test_conductive_state_stable_below_onset(glbm):
    print("case: onset, Ra = 0.8 x 1708", flush=True)
    s = _growth(glbm, 0.8 * 1708)
    print(f"growth rate {s:.3e} per step")
    assert s < 0


def test_conductive_state_unstable_above_onset(glbm):
    print("case: onset, Ra = 1.25 x 1708", flush=True)
    s = _growth(glbm, 1.25 * 1708)
    print(f"growth rate {s:.3e} per step")
    assert s > 0
