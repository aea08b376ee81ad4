"""GPU structure functions with horizontal increments (Fig. 3: S_2, S_4 and
the flatness of u_z and T) against the same averages of the FP64 oracle's
fields, on a state handed over through lbm_set_state (FP64 handle): agreement
to 1e-10 relative (the only difference is the order of FP64 sums)."""
import numpy as np
import pytest
import torch

import synth
from oracle import eos
from oracle import lbm as olbm

pytestmark = pytest.mark.gpu

TC = 0.05
KW = dict(tau_nu=0.8, tau_kappa=0.7, G=eos.coupling_for_tc(TC), T_d=0.95 * TC, T_u=0.85 * TC,
          gravity=1e-4)


@pytest.fixture(scope="module")
def glbm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1111_0905_amd import lbm
    lbm.load_library()
    return lbm


def _numpy_sf(a, rmax):
    s2, s4 = [], []
    for r in range(1, rmax + 1):
        dx = np.roll(a, -r, axis=2) - a
        dy = np.roll(a, -r, axis=1) - a
        d = np.concatenate([dx.ravel(), dy.ravel()])
        s2.append(np.mean(d ** 2))
        s4.append(np.mean(d ** 4))
    return np.array(s2), np.array(s4)


@pytest.mark.parametrize("shape,k0,k1,rmax", [((24, 20, 10), 2, 8, 9), ((9, 13, 6), 0, 6, 5)])
def test_structure_functions_match_oracle(glbm, shape, k0, k1, rmax):
    nx, ny, nz = shape
    p = olbm.Params(nx, ny, nz, **KW)
    o = olbm.Oracle(p, synth.noisy_density(nx, ny, nz, 1.3, 0.3, 31))
    o.step(30)
    m = o.fields()
    gp = glbm.Params(nx, ny, nz, storage=glbm.LBM_FP64, **KW)
    lat = glbm.Lattice(gp, torch.full((nx * ny * nz,), 1.3, dtype=torch.float64, device="cuda"))
    lat.set_state(o.state().cuda())
    for q, field in ((glbm.LBM_Q_VZ, m["v"][2]), (glbm.LBM_Q_T, m["T"])):
        a = field.numpy()[k0:k1]
        w2, w4 = _numpy_sf(a, rmax)
        g2, g4 = lat.structure_functions(k0, k1, q, rmax)
        assert np.abs(g2 - w2).max() <= 1e-10 * np.abs(w2).max()
        assert np.abs(g4 - w4).max() <= 1e-10 * np.abs(w4).max()


@pytest.mark.parametrize("storage", ["fp32", "fp16dev"])
def test_structure_functions_of_library_stepped_reduced_storage(glbm, storage):
    """FP32 and FP16-deviation handles stepped by the library: S_2, S_4 of
    u_z and T against the same averages of the handle's own moment fields
    (1e-10), and S_2 of T against the oracle's (the increments of T carry
    the fields' relative error times T / delta T: bars 1e-5 FP32, 2e-4 FP16;
    measured 5.9e-7 and 2.7e-5)."""
    nx, ny, nz = 24, 20, 10
    rho0 = synth.noisy_density(nx, ny, nz, 1.3, 0.3, 31)
    st = glbm.LBM_FP32 if storage == "fp32" else glbm.LBM_FP16DEV
    lat = glbm.Lattice(glbm.Params(nx, ny, nz, storage=st, rho_ref=1.3, T_ref=0.9 * TC, **KW),
                       torch.from_numpy(rho0).cuda())
    lat.step(30)
    _, fl = lat.fields()
    fl = fl.cpu().numpy()
    k0, k1, rmax = 2, 8, 9
    for q, field in ((glbm.LBM_Q_VZ, fl[3]), (glbm.LBM_Q_T, fl[4])):
        w2, w4 = _numpy_sf(field[k0:k1], rmax)
        g2, g4 = lat.structure_functions(k0, k1, q, rmax)
        assert np.abs(g2 - w2).max() <= 1e-10 * np.abs(w2).max()
        assert np.abs(g4 - w4).max() <= 1e-10 * np.abs(w4).max()
    o = olbm.Oracle(olbm.Params(nx, ny, nz, **KW), rho0).step(30)
    o2, _ = _numpy_sf(o.fields()["T"].numpy()[k0:k1], rmax)
    g2, _ = lat.structure_functions(k0, k1, glbm.LBM_Q_T, rmax)
    err = float(np.abs(g2 - o2).max() / np.abs(o2).max())
    print(f"{storage}: S_2(T) vs oracle {err:.2e}")
    assert err < (1e-5 if storage == "fp32" else 2e-4)


def test_structure_function_arguments(glbm):
    n = 8
    p = glbm.Params(n, n, n, storage=glbm.LBM_FP32, **KW)
    lat = glbm.Lattice(p, torch.full((n ** 3,), 1.3, dtype=torch.float64, device="cuda"))
    s2, s4 = lat.structure_functions(0, n, glbm.LBM_Q_T, 3)
    assert s2.shape == (3,) and np.all(s2 >= 0) and np.all(s4 >= 0)
    with pytest.raises(glbm.LbmError):
        lat.structure_functions(0, n, glbm.LBM_Q_T, n)      # r_max must stay below nx
    with pytest.raises(glbm.LbmError):
        lat.structure_functions(3, 3, glbm.LBM_Q_T, 2)
