"""MI355X (gfx950) implementation of the per-step sweep of the thermal
pseudopotential D3Q19 lattice Boltzmann scheme of arXiv:1111.0905.

The compute path is the HIP library `_lib/liblbm.so` (C ABI in
include/lbm.h); `paper_1111_0905_amd.lbm` is its ctypes binding, with torch
providing device memory and the stream.
"""
from .lbm import (  # noqa: F401
    LBM_BF16DEV, LBM_FP16DEV, LBM_FP32, LBM_FP64, LBM_KERNEL_FUSED, LBM_KERNEL_FUSED_RELOAD,
    LBM_KERNEL_REFERENCE, LbmError, Lattice, Params, lbm_destroy, lbm_get_state, lbm_init,
    lbm_histogram, lbm_moments, lbm_nusselt, lbm_seeded_density, lbm_set_state, lbm_step,
    lbm_structure_functions,
    lbm_time, lbm_workspace_bytes,
    load_library,
)
