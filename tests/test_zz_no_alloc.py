"""The allocation-free entry point lbm_structure_functions_noalloc (static
device scratch) against lbm_structure_functions (caller's work buffer),
through the C ABI: the same kernels on the same state give the same results
bit for bit, on two calls in a row, the second over fewer planes and a
smaller r_max; a request beyond the static scratch is refused."""
import ctypes

import numpy as np
import pytest
import torch

import synth
from oracle import eos

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


def _with_work(lib, lat, k0, k1, q, rmax):
    nb = lib.lbm_structure_work_bytes(lat.h.h, k0, k1, rmax)
    work = torch.empty(nb // 8 + 1, dtype=torch.float64, device="cuda")
    out = (ctypes.c_double * (2 * rmax))()
    rc = lib.lbm_structure_functions(lat.h.h, k0, k1, q, rmax, ctypes.c_void_p(work.data_ptr()),
                                     nb, out)
    assert rc == 0, lib.lbm_last_error()
    return np.array(out[:])


def _noalloc(lib, lat, k0, k1, q, rmax):
    out = (ctypes.c_double * (2 * rmax))()
    rc = lib.lbm_structure_functions_noalloc(lat.h.h, k0, k1, q, rmax, out)
    assert rc == 0, lib.lbm_last_error()
    return np.array(out[:])


@pytest.mark.parametrize("storage", ["fp32", "fp16dev"])
def test_noalloc_matches_work_buffer_entry_point(glbm, storage):
    lib = glbm.load_library()
    nx, ny, nz = 48, 40, 12
    rho0 = synth.noisy_density(nx, ny, nz, 1.3, 0.3, 31)
    st = glbm.LBM_FP32 if storage == "fp32" else glbm.LBM_FP16DEV
    lat = glbm.Lattice(glbm.Params(nx, ny, nz, storage=st, rho_ref=1.3, T_ref=0.9 * TC, **KW),
                       torch.from_numpy(rho0).cuda())
    lat.step(25)
    for k0, k1, rmax in ((1, 11, 17), (4, 6, 5)):     # the second call is smaller
        for q in (glbm.LBM_Q_VZ, glbm.LBM_Q_T):
            print(f"case: {storage} planes {k0}..{k1} r_max {rmax} q {q}", flush=True)
            a = _noalloc(lib, lat, k0, k1, q, rmax)
            b = _with_work(lib, lat, k0, k1, q, rmax)
            assert np.array_equal(a, b)
            assert np.all(a > 0)


def test_noalloc_refuses_more_than_its_scratch(glbm):
    lib = glbm.load_library()
    n = 256
    lat = glbm.Lattice(glbm.Params(n, n, 64, storage=glbm.LBM_FP32, **KW),
                       torch.full((n * n * 64,), 1.3, dtype=torch.float64, device="cuda"))
    out = (ctypes.c_double * 8)()
    assert lib.lbm_structure_functions_noalloc(lat.h.h, 0, 64, glbm.LBM_Q_T, 4, out) == -2
    assert b"static scratch" in lib.lbm_last_error()
    assert lib.lbm_structure_functions_noalloc(lat.h.h, 0, 32, glbm.LBM_Q_T, 4, out) == 0
