"""GPU histograms of node quantities (Fig. 2: the T-rho joint distribution of
the top panel, the pdf of the bulk heat flux rho U u_z in the inset of the
bottom panel) against the same binning of the FP64 oracle's fields.

The GPU gets the oracle's state through lbm_set_state on an FP64 handle, so
both sides bin the same values up to the rounding order of the node sums;
counts must agree exactly except for nodes that lie within 1e-9 of a bin
edge (in bin units), which may fall on either side.
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
KW = dict(tau_nu=0.8, tau_kappa=0.7, G=G, T_d=0.95 * TC, T_u=0.85 * TC, gravity=1e-4)


@pytest.fixture(scope="module")
def glbm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1111_0905_amd import lbm
    lbm.load_library()
    return lbm


@pytest.fixture(scope="module")
def state():
    nx, ny, nz = 20, 14, 12
    p = olbm.Params(nx, ny, nz, **KW)
    o = olbm.Oracle(p, synth.noisy_density(nx, ny, nz, 1.3, 0.3, 77))
    o.step(40)
    m = o.fields()
    U = olbm.internal_energy(p, m["rho"], m["T"])
    q = m["rho"] * U * m["v"][2]
    return (nx, ny, nz), o.state(), {"rho": m["rho"].numpy(), "T": m["T"].numpy(),
                                     "vz": m["v"][2].numpy(), "q": q.numpy()}


def _bins(x, lo, hi, n):
    f = (x - lo) * (n / (hi - lo))
    ok = (f >= 0) & (f < n)
    near = np.abs(f - np.round(f)) < 1e-9
    return np.floor(f).astype(np.int64), ok, near


def _gpu_lattice(glbm, shape, st):
    nx, ny, nz = shape
    p = glbm.Params(nx, ny, nz, storage=glbm.LBM_FP64, **KW)
    lat = glbm.Lattice(p, torch.full((nz * ny * nx,), 1.3, dtype=torch.float64, device="cuda"))
    lat.set_state(st.cuda())
    return lat


@pytest.mark.parametrize("k0,k1", [(0, 12), (3, 9)])
def test_joint_rho_T_histogram(glbm, state, k0, k1):
    shape, st, f = state
    lat = _gpu_lattice(glbm, shape, st)
    rr, tr, nb = (0.2, 2.6), (0.84 * TC, 0.96 * TC), (37, 23)
    counts, oor, sums = lat.histogram(k0, k1, glbm.LBM_Q_RHO, rr, nb[0], glbm.LBM_Q_T, tr, nb[1])
    rho, T = f["rho"][k0:k1].ravel(), f["T"][k0:k1].ravel()
    bx, okx, nx_ = _bins(rho, *rr, nb[0])
    by, oky, ny_ = _bins(T, *tr, nb[1])
    ok = okx & oky
    want = np.zeros(nb, dtype=np.int64)
    np.add.at(want, (bx[ok], by[ok]), 1)
    got = counts.cpu().numpy()
    ambiguous = int((nx_ | ny_).sum())
    assert np.abs(got - want).sum() <= 2 * ambiguous
    assert got.sum() + oor == rho.size
    assert sums[0] == rho.size
    assert abs(sums[1] - rho.sum()) < 1e-12 * rho.size
    assert abs(sums[3] - T.sum()) < 1e-12 * T.size
    assert abs(sums[2] - (rho ** 2).sum()) < 1e-12 * rho.size * 10


def test_bulk_heat_flux_pdf(glbm, state):
    shape, st, f = state
    lat = _gpu_lattice(glbm, shape, st)
    k0, k1 = 3, 9
    q = f["q"][k0:k1].ravel()
    lo, hi, n = float(q.min()) * 0.9, float(q.max()) * 0.9, 50
    counts, oor, sums = lat.histogram(k0, k1, glbm.LBM_Q_HEATFLUX, (lo, hi), n)
    b, ok, near = _bins(q, lo, hi, n)
    want = np.bincount(b[ok], minlength=n)
    got = counts.cpu().numpy().ravel()
    assert np.abs(got - want).sum() <= 2 * int(near.sum())
    assert oor == int((~ok).sum())
    assert abs(sums[1] - q.sum()) < 1e-9 * np.abs(q).sum()


def test_histogram_on_reduced_storage_counts_every_node(glbm):
    n = 16
    p = glbm.Params(n, n, n, storage=glbm.LBM_FP16DEV, rho_ref=1.3, T_ref=0.9 * TC, **KW)
    lat = glbm.Lattice(p, torch.from_numpy(synth.noisy_density(n, n, n, 1.3, 0.3, 5)).cuda())
    lat.step(10)
    counts, oor, sums = lat.histogram(0, n, glbm.LBM_Q_RHO, (0.5, 2.0), 64, glbm.LBM_Q_VZ,
                                      (-1e-3, 1e-3), 8)
    assert counts.sum().item() + oor == n ** 3 == sums[0]
    with pytest.raises(glbm.LbmError):
        lat.histogram(5, 5, glbm.LBM_Q_RHO, (0.5, 2.0), 8)
    with pytest.raises(glbm.LbmError):
        lat.histogram(0, n, glbm.LBM_Q_RHO, (2.0, 0.5), 8)
    with pytest.raises(glbm.LbmError):
        lat.histogram(0, n, 7, (0.5, 2.0), 8)


@pytest.mark.parametrize("storage", ["fp32", "fp16dev"])
def test_histograms_of_library_stepped_reduced_storage(glbm, storage):
    """FP32 and FP16-deviation handles stepped by the library (not loaded
    from the oracle): the joint (rho, T) histogram and the heat-flux pdf
    against the same binning of the handle's own moment fields (exact up to
    nodes on bin edges), and those fields against the oracle's within the
    storage form's bar (1e-5 FP32, 2e-4 FP16)."""
    nx, ny, nz = 20, 14, 12
    rho0 = synth.noisy_density(nx, ny, nz, 1.3, 0.3, 77)
    st = glbm.LBM_FP32 if storage == "fp32" else glbm.LBM_FP16DEV
    lat = glbm.Lattice(glbm.Params(nx, ny, nz, storage=st, rho_ref=1.3, T_ref=0.9 * TC, **KW),
                       torch.from_numpy(rho0).cuda())
    lat.step(40)
    _, fl = lat.fields()
    fl = fl.cpu().numpy()
    o = olbm.Oracle(olbm.Params(nx, ny, nz, **KW), rho0).step(40)
    m = o.fields()
    bar = 1e-5 if storage == "fp32" else 2e-4
    for a, b in ((fl[0], m["rho"].numpy()), (fl[4], m["T"].numpy())):
        assert np.abs(a - b).max() / np.abs(b).max() < bar
    k0, k1 = 0, nz
    rr, tr, nb = (0.2, 2.6), (0.84 * TC, 0.96 * TC), (37, 23)
    counts, oor, sums = lat.histogram(k0, k1, glbm.LBM_Q_RHO, rr, nb[0], glbm.LBM_Q_T, tr, nb[1])
    rho, T = fl[0][k0:k1].ravel(), fl[4][k0:k1].ravel()
    bx, okx, nx_ = _bins(rho, *rr, nb[0])
    by, oky, ny_ = _bins(T, *tr, nb[1])
    ok = okx & oky
    want = np.zeros(nb, dtype=np.int64)
    np.add.at(want, (bx[ok], by[ok]), 1)
    got = counts.cpu().numpy()
    assert np.abs(got - want).sum() <= 2 * int((nx_ | ny_).sum())
    assert got.sum() + oor == rho.size
    # heat-flux pdf: rho U v_z with U = c_v T + (G/4) exp(-2/rho)
    p = olbm.Params(nx, ny, nz, **KW)
    q = (fl[0] * (p.c_v * fl[4] + 0.25 * p.G * np.exp(-2.0 / fl[0])) * fl[3])[3:9].ravel()
    lo, hi, n = float(q.min()) * 0.9, float(q.max()) * 0.9, 50
    counts, oor, sums = lat.histogram(3, 9, glbm.LBM_Q_HEATFLUX, (lo, hi), n)
    b, okq, near = _bins(q, lo, hi, n)
    want = np.bincount(b[okq], minlength=n)
    assert np.abs(counts.cpu().numpy().ravel() - want).sum() <= 2 * int(near.sum())
    assert abs(sums[1] - q.sum()) < 1e-9 * np.abs(q).sum()
