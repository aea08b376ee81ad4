"""GPU parity of the pipelined step kernel (LBM_KERNEL_PIPELINED) against
the FP64 oracle, through the C ABI.

The pipelined kernel computes the same step as the other kernels with the
arithmetic reorganised (equilibria per pair of opposite directions, the
16-bit forms in deviation space, the force through grad(E - T_lat rho)), so
it is held to the storage form's bar against the oracle, not to bitwise
agreement with the other kernels.  Its tile shape and z chunking only change
which work-group computes a node, not how, so those variants must agree bit
for bit with each other.

Bars (relative to the field scale, after the stated steps): FP32 1e-5 on rho,
T and v; FP16 deviations 2e-4; BF16 deviations 2e-3 (as the packed-storage
parity tests of the other kernels).
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
BARS = {"fp32": 1e-5, "fp16dev": 2e-4, "bf16dev": 2e-3}


@pytest.fixture(scope="module")
def glbm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1111_0905_amd import lbm
    lbm.load_library()
    return lbm


def _kw(**over):
    kw = dict(tau_nu=1.0, tau_kappa=1.0, G=G, T_d=0.95 * TC, T_u=0.85 * TC, gravity=1e-5)
    kw.update(over)
    return kw


def _mean_density():
    rg, rl, _ = eos.maxwell(0.9 * TC, G)
    return 0.5 * (rg + rl)


def _oracle(nx, ny, nz, rho0, steps, **kw):
    periodic = kw.pop("periodic_z", 0)
    o = olbm.Oracle(olbm.Params(nx, ny, nz, periodic_z=bool(periodic), **kw), rho0)
    o.step(steps)
    return o


def _storage(glbm, name):
    return {"fp32": glbm.LBM_FP32, "fp16dev": glbm.LBM_FP16DEV, "bf16dev": glbm.LBM_BF16DEV}[name]


def _gpu(glbm, nx, ny, nz, rho0, steps, storage, **kw):
    p = glbm.Params(nx, ny, nz, storage=storage, kernel=glbm.LBM_KERNEL_PIPELINED, **kw)
    lat = glbm.Lattice(p, torch.from_numpy(np.ascontiguousarray(rho0)).cuda())
    lat.step(steps)
    torch.cuda.synchronize()
    return lat


def _rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def _field_errors(lat, o):
    _, fl = lat.fields()
    fl = fl.cpu().numpy()
    of = o.fields()
    v = of["v"].numpy()
    return (_rel(fl[0], of["rho"].numpy()), float(np.abs(fl[1:4] - v).max() / np.abs(v).max()),
            _rel(fl[4], of["T"].numpy()))


def test_config1_fp32_pipelined_matches_oracle(glbm):
    """32^3, walls, gravity, spinodal mean density, 100 steps (the parity
    configuration of the fused kernel)."""
    n = 32
    print("case: pipelined 32^3 FP32 100 steps", flush=True)
    rho0 = synth.noisy_density(n, n, n, _mean_density(), 0.01, 1234)
    o = _oracle(n, n, n, rho0, 100, **_kw())
    lat = _gpu(glbm, n, n, n, rho0, 100, glbm.LBM_FP32, **_kw())
    e_rho, e_v, e_T = _field_errors(lat, o)
    print(f"FP32 pipelined: rho {e_rho:.2e} v {e_v:.2e} T {e_T:.2e}")
    assert e_rho < BARS["fp32"] and e_v < BARS["fp32"] and e_T < BARS["fp32"]


@pytest.mark.parametrize("storage", ["fp32", "fp16dev", "bf16dev"])
@pytest.mark.parametrize("shape,periodic", [((65, 9, 13), 0), ((3, 17, 5), 0), ((130, 33, 4), 0),
                                            ((40, 20, 7), 1), ((24, 10, 1), 1), ((33, 17, 2), 0)])
def test_ragged_shapes_pipelined(glbm, storage, shape, periodic):
    """Partial tiles in x and y, few planes, periodic z (also a single
    plane), 20 steps against the oracle."""
    nx, ny, nz = shape
    print(f"case: pipelined ragged {shape} periodic={periodic} {storage}", flush=True)
    rho_m = _mean_density()
    rho0 = synth.noisy_density(nx, ny, nz, rho_m, 0.02, 31)
    kw = _kw(tau_nu=0.8, tau_kappa=0.7, gravity=1e-4, periodic_z=periodic)
    o = _oracle(nx, ny, nz, rho0, 20, **kw)
    lat = _gpu(glbm, nx, ny, nz, rho0, 20, _storage(glbm, storage), rho_ref=rho_m,
               T_ref=0.9 * TC, **kw)
    e_rho, e_v, e_T = _field_errors(lat, o)
    print(f"{storage} {shape}: rho {e_rho:.2e} v {e_v:.2e} T {e_T:.2e}")
    bar = BARS[storage]
    assert e_rho < bar and e_T < bar


@pytest.mark.parametrize("storage", ["fp32", "fp16dev"])
def test_tiles_and_chunks_bit_identical(glbm, storage):
    """Every tile shape and z chunking of the pipelined kernel gives the same
    state bit for bit (70 x 19 x 23, walls, 7 steps)."""
    nx, ny, nz = 70, 19, 23
    rho0 = synth.noisy_density(nx, ny, nz, 1.9, 0.05, 11)
    kw = _kw(tau_nu=0.7, tau_kappa=0.9, gravity=1e-4)
    ref = None
    for tx, ty, zc in [(32, 16, 0), (32, 16, 1), (32, 16, 2), (32, 16, 5), (32, 8, 0),
                       (64, 8, 3), (16, 16, 0), (16, 16, 4), (32, 16, 23), (128, 4, 0),
                       (256, 2, 0), (256, 2, 6)]:
        print(f"case: pipelined {storage} tile {tx}x{ty} z_chunk={zc}", flush=True)
        lat = _gpu(glbm, nx, ny, nz, rho0, 7, _storage(glbm, storage), tile_x=tx, tile_y=ty,
                   z_chunk=zc, rho_ref=1.9, T_ref=0.9 * TC, **kw)
        s = lat.state().cpu()
        if ref is None:
            ref = s
        else:
            assert torch.equal(s, ref), (tx, ty, zc)


@pytest.mark.parametrize("storage", ["fp32", "fp16dev"])
def test_default_launch_shape_bit_identical(glbm, storage):
    """512 x 516 x 16 with the default 128 x 4 tiles: 516 tiles, three rounds of
    the GPU's 256 resident work-groups if the column is not split, and not a
    multiple of 8.  The default z chunking (which splits the 16 planes in
    two: 1032 work-groups), one chunk (516 work-groups, so the XCD tile map
    takes its uneven form) and 4-plane chunks give the same state bit for
    bit after 3 steps."""
    nx, ny, nz = 512, 516, 16
    rho0 = synth.noisy_density(nx, ny, nz, 1.9, 0.05, 12)
    kw = _kw(tau_nu=0.7, tau_kappa=0.9, gravity=1e-4)
    ref = None
    for zc in (0, 16, 4):
        print(f"case: pipelined {storage} {nx}x{ny}x{nz} z_chunk={zc}", flush=True)
        lat = _gpu(glbm, nx, ny, nz, rho0, 3, _storage(glbm, storage), z_chunk=zc, rho_ref=1.9,
                   T_ref=0.9 * TC, **kw)
        s = lat.state()
        if ref is None:
            ref = s.clone()
        else:
            assert torch.equal(s, ref), zc
        del lat, s
        torch.cuda.empty_cache()


@pytest.mark.parametrize("storage", ["fp32", "fp16dev"])
def test_variants_pipelined(glbm, storage):
    """Wetting walls with the original Shan-Chen pseudopotential, and the
    force-form coupling T_lat = 1/3: 20 x 12 x 16, 60 steps."""
    nx, ny, nz = 20, 12, 16
    rg, rl, _ = eos.maxwell(0.9 * TC, G)
    cases = [("wetting", _kw(rho_wall_d=rl, rho_wall_u=rg), _mean_density()),
             ("shan-chen", _kw(G=-4 * TC, psi_form=1, rho_wall_d=1.5), 1.0),
             ("force-form", _kw(T_lat=1.0 / 3.0), _mean_density())]
    for name, kw, rho_m in cases:
        print(f"case: pipelined {storage} {name}", flush=True)
        rho0 = synth.noisy_density(nx, ny, nz, rho_m, 0.02, 77)
        o = _oracle(nx, ny, nz, rho0, 60, **kw)
        lat = _gpu(glbm, nx, ny, nz, rho0, 60, _storage(glbm, storage), rho_ref=rho_m,
                   T_ref=0.9 * TC, **kw)
        e_rho, e_v, e_T = _field_errors(lat, o)
        print(f"{storage} {name}: rho {e_rho:.2e} v {e_v:.2e} T {e_T:.2e}")
        assert e_rho < BARS[storage] and e_T < BARS[storage]


@pytest.mark.parametrize("storage", ["fp32", "fp16dev", "bf16dev"])
def test_mass_conserved_pipelined(glbm, storage):
    """Periodic 32^3 box at the spinodal density (phase separation from 5 %
    noise), 300 steps: the stored mass, summed in FP64 from the stored words,
    moves only by roundings that are not correlated between nodes.  Every
    node adds its remainder sum to its FP32 rest population once per step; in
    this violent run that sum is non-zero everywhere, so each add rounds by a
    uniform error of rms ulp(f_0)/sqrt(12) (f_0 ~ 1.1, ulp 2^-23): over N
    nodes and s steps a random walk of rms sqrt(N s) ulp/sqrt(12) / M ~ 3e-9
    relative.  Bar: 5 times that (1.5e-8) for the 16-bit forms; FP32 storage
    also rounds every collided population to FP32 (bar 1e-7, as for the other
    kernels).  (Runs near equilibrium, where the quantised populations stop
    changing, conserve far better: the remainder sums vanish.)"""
    n = 32
    rho_m = _mean_density()
    rho0 = synth.noisy_density(n, n, n, rho_m, 0.05, 5)
    print(f"case: pipelined mass {storage}", flush=True)
    lat = _gpu(glbm, n, n, n, rho0, 0, _storage(glbm, storage), periodic_z=1, gravity=0.0,
               rho_ref=rho_m, T_ref=0.9 * TC, **{k: v for k, v in _kw().items() if k != "gravity"})
    m0 = lat.moments()[0]
    lat.step(300)
    m1 = lat.moments()[0]
    drift = abs(m1 / m0 - 1)
    print(f"{storage}: mass drift {drift:.2e}")
    assert drift < (1e-7 if storage == "fp32" else 1.5e-8)
