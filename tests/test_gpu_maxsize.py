"""Parity at the largest lattice the library accepts: 812^3 nodes, where one
population row of the FP32 and 16-bit forms (8 B per node) is just under
4 GiB, so the 32-bit node and byte offsets of the kernels are at their limit
(813^3 is refused, see the ABI test).  4 steps of a walled, gravity-driven
cell at the spinodal mean density from seeded noise; sampled full-height
columns, including ones on the last x and y indices, against the FP64 oracle
stepping a (4 s + 1)^2 x 812 patch around each (the domain-of-dependence
argument of the full-size test).  Needs about 200 GB of device memory for
FP32; skipped on smaller devices.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import eos
from oracle import lbm as olbm

pytestmark = pytest.mark.gpu

N = 812
STEPS = 4
HALF = 2 * STEPS
TC = 0.05
G = eos.coupling_for_tc(TC)
SEED, AMP = 1234, 0.01
COLUMNS = [(0, 0), (N - 1, 5), (405, N - 1), (N - 1, N - 1)]
BARS = {"fp32": (1e-5, 2e-6), "fp16dev": (1e-4, 1e-5)}
KW = dict(tau_nu=1.0, tau_kappa=1.0, G=G, T_d=0.95 * TC, T_u=0.85 * TC, gravity=1e-5)


@pytest.fixture(scope="module")
def glbm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    free, _ = torch.cuda.mem_get_info()
    if free < 210 * 2 ** 30:
        pytest.skip("needs about 200 GB of free device memory")
    from paper_1111_0905_amd import lbm
    lbm.load_library()
    return lbm


def _rho_mean():
    rg, rl, _ = eos.maxwell(0.9 * TC, G)
    return 0.5 * (rg + rl)


@pytest.fixture(scope="module")
def oracle_columns():
    rho_m = _rho_mean()
    po = olbm.Params(2 * HALF + 1, 2 * HALF + 1, N, **KW)
    out = {}
    for (x, y) in COLUMNS:
        xs = np.array([(x + d) % N for d in range(-HALF, HALF + 1)])
        ys = np.array([(y + d) % N for d in range(-HALF, HALF + 1)])
        ks = np.arange(N)
        patch = synth.noisy_density_at(N, N, N, rho_m, AMP, SEED, ks[:, None, None],
                                       ys[None, :, None], xs[None, None, :])
        o = olbm.Oracle(po, np.ascontiguousarray(patch))
        o.step(STEPS)
        m = o.fields()
        out[(x, y)] = (m["rho"][:, HALF, HALF].numpy(), m["v"][:, :, HALF, HALF].numpy(),
                       m["T"][:, HALF, HALF].numpy())
    return out


@pytest.mark.parametrize("storage", ["fp32", "fp16dev"])
def test_largest_lattice_sampled_columns(glbm, oracle_columns, storage):
    print(f"case: {N}^3 {storage}, {STEPS} steps", flush=True)
    rho_m = _rho_mean()
    st = {"fp32": glbm.LBM_FP32, "fp16dev": glbm.LBM_FP16DEV}[storage]
    p = glbm.Params(N, N, N, storage=st, rho_ref=rho_m, T_ref=0.9 * TC, **KW)
    rho0 = glbm.lbm_seeded_density(N, N, N, SEED, rho_m, AMP).reshape(-1)
    lat = glbm.Lattice(p, rho0)
    del rho0
    lat.step(STEPS)
    _, fl = lat.fields()
    cols = {c: fl[:, :, c[1], c[0]].cpu().numpy() for c in COLUMNS}
    tot = lat.moments()
    del fl, lat
    torch.cuda.empty_cache()
    assert np.isfinite(tot).all()
    b_s, b_v = BARS[storage]
    worst = [0.0, 0.0, 0.0]
    for c in COLUMNS:
        rho, v, T = oracle_columns[c]
        g = cols[c]
        e = [float(np.abs(g[0] - rho).max() / np.abs(rho).max()),
             float(np.abs(g[1:4] - v).max()),
             float(np.abs(g[4] - T).max() / np.abs(T).max())]
        worst = [max(a, b) for a, b in zip(worst, e)]
    print(f"{storage}: worst rho {worst[0]:.2e} T {worst[2]:.2e} (relative), v {worst[1]:.2e}")
    assert worst[0] < b_s and worst[2] < b_s
    assert worst[1] < b_v
