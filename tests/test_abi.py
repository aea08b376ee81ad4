"""The C-ABI library loads and exports every entry point include/lbm.h
declares; host-side parameter validation works without a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    from paper_1111_0905_amd import lbm
    return lbm.load_library()


def test_header_declares_the_boundary():
    names = _declared()
    for want in ["lbm_init", "lbm_step", "lbm_moments", "lbm_nusselt", "lbm_get_state",
                 "lbm_set_state", "lbm_workspace_bytes", "lbm_destroy", "lbm_last_error"]:
        assert want in names


def test_library_exports_every_declared_symbol(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def test_version_string(lib):
    assert b"gfx950" in lib.lbm_version()


def test_workspace_bytes_and_validation(lib):
    from paper_1111_0905_amd import lbm
    p = lbm.Params(64, 32, 16, storage=lbm.LBM_FP32)
    n = p.n
    nb = lbm.lbm_workspace_bytes(p)
    assert nb >= 2 * 38 * n * 4 + 2 * n * 4
    p64 = lbm.Params(64, 32, 16, storage=lbm.LBM_FP64)
    assert lbm.lbm_workspace_bytes(p64) > nb
    p16 = lbm.Params(64, 32, 16, storage=lbm.LBM_FP16DEV)
    assert lbm.lbm_workspace_bytes(p16) < nb
    for bad in [dict(nx=0), dict(tau_nu=0.5), dict(tau_kappa=0.3), dict(G=0.1), dict(T_d=0.0),
                dict(nz=1), dict(storage=7), dict(kernel=9), dict(c_v=0.0), dict(tile_y=3),
                dict(storage=lbm.LBM_FP16DEV, rho_ref=0.0), dict(psi_form=2),
                dict(rho_wall_d=float("nan"))]:
        q = lbm.Params(8, 8, 8)
        for k, v in bad.items():
            setattr(q, k, v)
        with pytest.raises(lbm.LbmError):
            lbm.lbm_workspace_bytes(q)
    # one plane is fine without walls
    assert lbm.lbm_workspace_bytes(lbm.Params(8, 8, 1, periodic_z=1)) > 0


def test_null_handle_is_rejected(lib):
    assert lib.lbm_step(None, 1) == -1
    assert b"NULL" in lib.lbm_last_error()


def test_largest_lattices(lib):
    """Every direction's array must stay below 4 GiB (32-bit node offsets):
    the widest row holds 8 B per node in FP32 and the 16-bit forms (their
    FP32 rest pair) and 16 B in FP64."""
    from paper_1111_0905_amd import lbm
    assert lbm.lbm_workspace_bytes(lbm.Params(812, 812, 812, storage=lbm.LBM_FP32)) > 0
    with pytest.raises(lbm.LbmError):
        lbm.lbm_workspace_bytes(lbm.Params(813, 813, 813, storage=lbm.LBM_FP32))
    assert lbm.lbm_workspace_bytes(lbm.Params(812, 812, 812, storage=lbm.LBM_FP16DEV,
                                              rho_ref=1.0, T_ref=0.05)) > 0
    assert lbm.lbm_workspace_bytes(lbm.Params(645, 645, 645, storage=lbm.LBM_FP64)) > 0
    with pytest.raises(lbm.LbmError):
        lbm.lbm_workspace_bytes(lbm.Params(646, 646, 646, storage=lbm.LBM_FP64))
    # 16-bit forms: 80 B per node and buffer (FP32 rest pair + 18 words)
    w16 = lbm.lbm_workspace_bytes(lbm.Params(512, 512, 512, storage=lbm.LBM_FP16DEV,
                                             rho_ref=1.0, T_ref=0.05))
    assert w16 >= 2 * 80 * 512 ** 3


def test_null_arguments_of_diagnostics(lib):
    assert lib.lbm_histogram(None, 0, 1, 0, 0.0, 1.0, 1, -1, 0.0, 1.0, 1, None, None, None) == -1
    assert lib.lbm_seeded_density(4, 4, 4, 1, 1.0, 0.1, None, None) == -1
    assert lib.lbm_structure_work_bytes(None, 0, 1, 1) == 0


def test_pipelined_kernel_validation(lib):
    from paper_1111_0905_amd import lbm
    ok = lbm.Params(64, 32, 16, storage=lbm.LBM_FP16DEV, kernel=lbm.LBM_KERNEL_PIPELINED,
                    tile_x=128, tile_y=4)
    assert lbm.lbm_workspace_bytes(ok) > 0
    for bad in [dict(storage=lbm.LBM_FP64), dict(tile_x=64, tile_y=16), dict(tile_x=32, tile_y=32)]:
        kw = dict(storage=lbm.LBM_FP32, kernel=lbm.LBM_KERNEL_PIPELINED)
        kw.update(bad)
        with pytest.raises(lbm.LbmError):
            lbm.lbm_workspace_bytes(lbm.Params(64, 32, 16, **kw))


def test_stream_references_reject_bad_arguments(lib):
    """Argument checks of the bandwidth references happen before any launch."""
    fake = ctypes.c_void_p(4096)
    assert lib.lbm_stream_copy(None, fake, 16, 0, None) == -1
    assert lib.lbm_stream_copy(fake, fake, 0, 0, None) == -1
    assert lib.lbm_stream_copy(fake, fake, 24, 0, None) == -1           # not a multiple of 16
    assert lib.lbm_stream_copy(ctypes.c_void_p(4104), fake, 32, 0, None) == -1   # misaligned
    assert lib.lbm_stream_rows(fake, fake, 3, 64, 64, None) == -1       # unsupported row count
    assert lib.lbm_stream_rows(fake, fake, 19, 32, 64, None) == -1      # stride < row bytes
    assert lib.lbm_stream_rows(fake, fake, 19, 64, 12, None) == -1      # not a multiple of 8
    assert b"rows" in lib.lbm_last_error() or b"row" in lib.lbm_last_error()
