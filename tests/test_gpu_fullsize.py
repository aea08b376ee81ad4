"""Parity at full size: the 512^3 boiling convection cell in the launch
configuration the throughput benchmark times (default kernel, tiles and
z-chunking for each storage form), and the 128^3 cell (whose default launch
runs the pipelined kernel on 128 x 4 tiles and splits the z columns into
16-plane chunks, so that one round of work-groups covers the lattice).

The oracle cannot step 512^3 nodes, but one node's state after s steps
depends only on the state within 2 s nodes of it in x and y (the force at a
neighbour needs psi, rho and E one node further; streaming moves one node),
and the walls in z; the velocity v = (j + F/2)/rho of that node also needs
the force, so one node more.  So for a few sampled (x, y) columns the oracle
steps a (4 s + 3) x (4 s + 3) x 512 patch cut from the same seeded initial
field (periodic across the patch, which disturbs only its outer 2 s + 1
nodes) and the centre column is compared with the GPU's, all 512 planes of
it.

Bars: relative on rho and T (field-scale metric: max |difference| over the
column / max |oracle value|): FP32 storage 1e-5, the 16-bit deviation forms
as in the small-grid precision tests.  Velocity: absolute, since four steps
from rest leave |v| ~ 1e-3, where the storage rounding of the populations
(unit roundoff times sum |f_l| ~ rho for FP32, times the deviations for the
16-bit forms) already decides the relative error.
"""
import numpy as np
import pytest
import torch

import bench
import synth
from oracle import lbm as olbm

pytestmark = pytest.mark.gpu

STEPS = 4
# a node's state after s steps depends on the states within 2 s nodes; its
# velocity v = (j + F/2)/rho also on the force, hence on one node more
HALF = 2 * STEPS + 1
BARS = {"fp32": (1e-5, 2e-6), "fp16dev": (1e-4, 1e-5), "bf16dev": (1e-3, 1e-4)}
CASES = {512: [(0, 0), (511, 7), (130, 511), (257, 300), (401, 64), (37, 255)],
         128: [(0, 0), (127, 5), (64, 127), (33, 90)]}


@pytest.fixture(scope="module")
def glbm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1111_0905_amd import lbm
    lbm.load_library()
    return lbm


def _params(lbm, n, storage):
    if n == 512:
        return bench.workload_params(lbm, n, storage)
    from paper_1111_0905_amd import experiments
    rho = experiments.boiling_density(n, 1e6)
    return experiments.cell_params(n, rho, 1e6, storage)


_cache = {}


def _field_and_oracle(n):
    if n in _cache:
        return _cache[n]
    from paper_1111_0905_amd import lbm
    p = _params(lbm, n, "fp32")
    rho0 = bench.seeded_density(n, p.rho_ref)      # (z, y, x)
    po = olbm.Params(2 * HALF + 1, 2 * HALF + 1, n, tau_nu=p.tau_nu, tau_kappa=p.tau_kappa,
                     G=p.G, T_d=p.T_d, T_u=p.T_u, gravity=p.gravity, c_v=p.c_v,
                     rho_kappa=p.rho_kappa, T_lat=p.T_lat)
    cols = {}
    for (x, y) in CASES[n]:
        xs = [(x + d) % n for d in range(-HALF, HALF + 1)]
        ys = [(y + d) % n for d in range(-HALF, HALF + 1)]
        patch = rho0[:, ys][:, :, xs]
        o = olbm.Oracle(po, np.ascontiguousarray(patch))
        o.step(STEPS)
        m = o.fields()
        cols[(x, y)] = (m["rho"][:, HALF, HALF].numpy(), m["v"][:, :, HALF, HALF].numpy(),
                        m["T"][:, HALF, HALF].numpy())
    _cache.clear()
    _cache[n] = (rho0, cols)
    return _cache[n]


@pytest.mark.parametrize("n", [512, 128])
@pytest.mark.parametrize("storage", ["fp32", "fp16dev", "bf16dev"])
def test_sampled_columns_match_oracle(glbm, n, storage):
    print(f"case: {n}^3 {storage}, benchmark launch configuration, {STEPS} steps", flush=True)
    rho0, oracle_columns = _field_and_oracle(n)
    p = _params(glbm, n, storage)
    lat = glbm.Lattice(p, torch.from_numpy(rho0).cuda().reshape(-1))
    lat.step(STEPS)
    _, fl = lat.fields()
    cols = {c: fl[:, :, c[1], c[0]].cpu().numpy() for c in CASES[n]}
    del fl, lat
    torch.cuda.empty_cache()
    b_s, b_v = BARS[storage]
    worst = [0.0, 0.0, 0.0]
    for c in CASES[n]:
        rho, v, T = oracle_columns[c]
        g = cols[c]
        e = [float(np.abs(g[0] - rho).max() / np.abs(rho).max()),
             float(np.abs(g[1:4] - v).max()),
             float(np.abs(g[4] - T).max() / np.abs(T).max())]
        worst = [max(a, b) for a, b in zip(worst, e)]
    vmax = max(float(np.abs(oracle_columns[c][1]).max()) for c in CASES[n])
    print(f"{storage}: worst rho {worst[0]:.2e} T {worst[2]:.2e} (relative), "
          f"v {worst[1]:.2e} (absolute; max |v| {vmax:.2e})")
    assert worst[0] < b_s and worst[2] < b_s
    assert worst[1] < b_v
