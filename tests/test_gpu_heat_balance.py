"""GPU parity of the pressure-work profile <P d_j u_j>(k), the right-hand
side of the layer heat balance eq. (heat2) and the integrand of the
constraint eq. (flux), against the FP64 oracle (whose profile is pinned by a
closed form and by the heat balance itself in test_oracle_diagnostics.py).

Bars: FP64 storage 1e-10 of the profile's largest magnitude (the profile
differences velocities, so the step's 1e-14 state agreement grows by the
inverse of the velocity scale); FP32 storage 2e-3 (velocity fields carry
~1e-5 relative error, which the divergence of a nearly solenoidal flow
amplifies).
"""
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


@pytest.mark.parametrize("storage", ["fp64", "fp32"])
@pytest.mark.parametrize("periodic", [0, 1])
def test_pressure_work_matches_oracle(glbm, storage, periodic):
    nx, ny, nz = 20, 12, 16
    rg, rl, _ = eos.maxwell(0.9 * TC, G)
    rho0 = synth.noisy_density(nx, ny, nz, 0.5 * (rg + rl), 0.03, 19)
    kw = dict(tau_nu=0.8, tau_kappa=0.7, G=G, T_d=0.95 * TC, T_u=0.85 * TC, gravity=1e-4)
    print(f"case: pressure work {storage} periodic={periodic}", flush=True)
    o = olbm.Oracle(olbm.Params(nx, ny, nz, periodic_z=bool(periodic), **kw), rho0).step(30)
    want = olbm.pressure_work(o.p, o.f, o.g).numpy()
    st = glbm.LBM_FP64 if storage == "fp64" else glbm.LBM_FP32
    lat = glbm.Lattice(glbm.Params(nx, ny, nz, storage=st, periodic_z=periodic, **kw),
                       torch.from_numpy(rho0).cuda())
    lat.step(30)
    got = lat.pressure_work()
    err = float(np.abs(got - want).max() / np.abs(want).max())
    print(f"{storage} periodic={periodic}: max |P div v| {np.abs(want).max():.3e}, rel err {err:.2e}")
    assert err < (1e-10 if storage == "fp64" else 2e-3)


def test_pressure_work_argument_checks(glbm):
    lat = glbm.Lattice(glbm.Params(8, 8, 4, storage=glbm.LBM_FP32), np.full((4, 8, 8), 1.5))
    out = (glbm.ctypes.c_double * 4)()
    work = torch.empty(5 * 8 * 8 * 4, dtype=torch.float64, device="cuda")
    lib = glbm.load_library()
    assert lib.lbm_pressure_work(lat.h.h, glbm.ctypes.c_void_p(work.data_ptr()), 8, out) == -2
    assert lib.lbm_pressure_work(lat.h.h, None, 5 * 256 * 8, out) == -1
