"""ctypes binding of the C ABI in include/lbm.h.

Argument marshalling only: every step of the lattice update runs in the HIP
kernels of _lib/liblbm.so.  torch provides the device workspace, the device
arrays handed across the boundary and the HIP stream.  There is no CPU
fallback: if the library is missing, loading fails loudly.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass, fields

import numpy as np

LBM_FP64, LBM_FP32, LBM_FP16DEV, LBM_BF16DEV = 0, 1, 2, 3
LBM_KERNEL_FUSED, LBM_KERNEL_REFERENCE, LBM_KERNEL_FUSED_RELOAD, LBM_KERNEL_PIPELINED = 0, 1, 2, 3
STORAGE = {"fp64": LBM_FP64, "fp32": LBM_FP32, "fp16dev": LBM_FP16DEV, "bf16dev": LBM_BF16DEV}
LBM_Q_RHO, LBM_Q_T, LBM_Q_VZ, LBM_Q_HEATFLUX = 0, 1, 2, 3

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_lib", "liblbm.so")
_lib = None


class LbmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"lbm error {code}: {msg}")
        self.code = code


class _CParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("storage", ctypes.c_int32), ("periodic_z", ctypes.c_int32), ("kernel", ctypes.c_int32),
        ("tile_x", ctypes.c_int32), ("tile_y", ctypes.c_int32), ("z_chunk", ctypes.c_int32),
        ("adjoint", ctypes.c_int32),
        ("tau_nu", ctypes.c_double), ("tau_kappa", ctypes.c_double), ("G", ctypes.c_double),
        ("T_d", ctypes.c_double), ("T_u", ctypes.c_double), ("gravity", ctypes.c_double),
        ("c_v", ctypes.c_double), ("rho_kappa", ctypes.c_double),
        ("rho_ref", ctypes.c_double), ("T_ref", ctypes.c_double), ("T_lat", ctypes.c_double),
        ("rho_wall_d", ctypes.c_double), ("rho_wall_u", ctypes.c_double),
        ("psi_form", ctypes.c_int32),
    ]


@dataclass
class Params:
    """Problem statement; field names follow include/lbm.h."""
    nx: int
    ny: int
    nz: int
    storage: int = LBM_FP32
    periodic_z: int = 0
    kernel: int = LBM_KERNEL_FUSED
    tile_x: int = 0
    tile_y: int = 0
    z_chunk: int = 0
    adjoint: int = 0
    tau_nu: float = 1.0
    tau_kappa: float = 1.0
    G: float = -0.05 * math.e ** 2
    T_d: float = 0.0475
    T_u: float = 0.0425
    gravity: float = 0.0
    c_v: float = 1.0
    rho_kappa: float = 0.5
    rho_ref: float = 1.0
    T_ref: float = 0.045
    T_lat: float = 0.0
    rho_wall_d: float = 0.0
    rho_wall_u: float = 0.0
    psi_form: int = 0

    def c(self) -> _CParams:
        return _CParams(**{f.name: getattr(self, f.name) for f in fields(self)})

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz


def load_library(path: str = _LIB_PATH):
    """Load liblbm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"HIP library {path} is missing: run __graft_entry__.build() first")
    lib = ctypes.CDLL(path)
    P, H, D = ctypes.POINTER(_CParams), ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)
    sig = {
        "lbm_version": ([], ctypes.c_char_p),
        "lbm_last_error": ([], ctypes.c_char_p),
        "lbm_workspace_bytes": ([P], ctypes.c_size_t),
        "lbm_init": ([P, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p,
                      ctypes.c_void_p, ctypes.POINTER(H)], ctypes.c_int),
        "lbm_step": ([H, ctypes.c_int64], ctypes.c_int),
        "lbm_set_check": ([H, ctypes.c_int64, ctypes.c_double], ctypes.c_int),
        "lbm_time": ([H], ctypes.c_int64),
        "lbm_moments": ([H, D, ctypes.c_void_p], ctypes.c_int),
        "lbm_nusselt": ([H, D, D, D, D], ctypes.c_int),
        "lbm_get_state": ([H, ctypes.c_void_p], ctypes.c_int),
        "lbm_set_state": ([H, ctypes.c_void_p], ctypes.c_int),
        "lbm_destroy": ([H], None),
        "lbm_adjoint_step": ([H, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, D], ctypes.c_int),
        "lbm_adjoint_qbot": ([H, ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p, D, D],
                             ctypes.c_int),
        "lbm_adjoint_init_rho": ([H, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p],
                                 ctypes.c_int),
        "lbm_seeded_density": ([ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64,
                                ctypes.c_double, ctypes.c_double, ctypes.c_void_p,
                                ctypes.c_void_p], ctypes.c_int),
        "lbm_structure_work_bytes": ([H, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32],
                                     ctypes.c_size_t),
        "lbm_structure_functions_noalloc": ([H, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                             ctypes.c_int32, D], ctypes.c_int),
        "lbm_structure_functions": ([H, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.c_int32, ctypes.c_void_p, ctypes.c_size_t, D],
                                    ctypes.c_int),
        "lbm_pressure_work": ([H, ctypes.c_void_p, ctypes.c_size_t, D], ctypes.c_int),
        "lbm_stream_copy": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32,
                             ctypes.c_void_p], ctypes.c_int),
        "lbm_stream_rows": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t,
                             ctypes.c_size_t, ctypes.c_void_p], ctypes.c_int),
        "lbm_histogram": ([H, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                           ctypes.c_double, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                           ctypes.c_double, ctypes.c_int32, ctypes.c_void_p,
                           ctypes.POINTER(ctypes.c_uint64), D], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _check(rc: int):
    if rc != 0:
        raise LbmError(rc, load_library().lbm_last_error().decode())


def _dev_ptr(t, dtype, numel):
    import torch
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous() or t.numel() != numel:
        raise ValueError(f"expected a contiguous {dtype} cuda tensor with {numel} elements")
    return ctypes.c_void_p(t.data_ptr())


def lbm_workspace_bytes(p: Params) -> int:
    cp = p.c()
    n = load_library().lbm_workspace_bytes(ctypes.byref(cp))
    if n == 0:
        raise LbmError(-1, load_library().lbm_last_error().decode())
    return n


class _Handle:
    """A lattice on the device: the C handle plus the torch-owned workspace."""

    def __init__(self, p: Params, h, workspace, stream):
        self.p, self.h, self.workspace, self.stream = p, h, workspace, stream

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.lbm_destroy(self.h)
            self.h = None


def lbm_init(p: Params, rho0, T0=None, stream=None) -> _Handle:
    """rho0 (and T0): torch float64 cuda tensors of nx*ny*nz elements."""
    import torch
    lib = load_library()
    nbytes = lbm_workspace_bytes(p)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=rho0.device)
    if ws.data_ptr() % 256:
        raise LbmError(-2, "torch workspace not 256-byte aligned")
    stream = stream if stream is not None else torch.cuda.current_stream(rho0.device)
    # the handle's work runs on `stream`: tell torch's caching allocator, so the
    # workspace is not handed out again before that work has finished
    ws.record_stream(stream)
    h = ctypes.c_void_p()
    cp = p.c()
    T0p = _dev_ptr(T0, torch.float64, p.n) if T0 is not None else None
    _check(lib.lbm_init(ctypes.byref(cp), ctypes.c_void_p(ws.data_ptr()), nbytes,
                        _dev_ptr(rho0, torch.float64, p.n), T0p,
                        ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h)))
    return _Handle(p, h, ws, stream)


def lbm_step(h: _Handle, n: int = 1):
    _check(load_library().lbm_step(h.h, int(n)))


def lbm_time(h: _Handle) -> int:
    return load_library().lbm_time(h.h)


def lbm_moments(h: _Handle, fields=None) -> np.ndarray:
    """Totals [M, Px, Py, Pz, sum rho T, sum rho U]; fields (optional) is a
    float64 cuda tensor of 5*N elements receiving rho, vx, vy, vz, T."""
    import torch
    tot = (ctypes.c_double * 6)()
    fp = _dev_ptr(fields, torch.float64, 5 * h.p.n) if fields is not None else None
    _check(load_library().lbm_moments(h.h, tot, fp))
    return np.array(tot[:], dtype=np.float64)


def lbm_nusselt(h: _Handle):
    """(nu_bot, nu_top, nu_z[nz], T_z[nz])."""
    nz = h.p.nz
    nb, nt = ctypes.c_double(), ctypes.c_double()
    nu_z = (ctypes.c_double * nz)()
    T_z = (ctypes.c_double * nz)()
    _check(load_library().lbm_nusselt(h.h, ctypes.byref(nb), ctypes.byref(nt), nu_z, T_z))
    return nb.value, nt.value, np.array(nu_z[:]), np.array(T_z[:])


def lbm_histogram(h: _Handle, k0: int, k1: int, qx: int, x_range, nx_bins: int, qy: int = -1,
                  y_range=(0.0, 1.0), ny_bins: int = 1):
    """(counts [nx_bins, ny_bins] int64 cuda tensor, out_of_range, sums[5]) over planes
    k0 <= k < k1; sums = [nodes, sum x, sum x^2, sum y, sum y^2]."""
    import torch
    counts = torch.empty((nx_bins, ny_bins), dtype=torch.int64, device=h.workspace.device)
    oor = ctypes.c_uint64()
    sums = (ctypes.c_double * 5)()
    _check(load_library().lbm_histogram(h.h, k0, k1, qx, float(x_range[0]), float(x_range[1]),
                                        nx_bins, qy, float(y_range[0]), float(y_range[1]),
                                        ny_bins, _dev_ptr(counts, torch.int64, nx_bins * ny_bins),
                                        ctypes.byref(oor), sums))
    return counts, oor.value, np.array(sums[:])


def lbm_seeded_density(nx: int, ny: int, nz: int, seed: int, rho_mean: float, noise_amp: float,
                       device="cuda", stream=None):
    """Seeded initial density (nz, ny, nx) float64 on the device (SplitMix64 per node)."""
    import torch
    out = torch.empty((nz, ny, nx), dtype=torch.float64, device=device)
    s = stream if stream is not None else torch.cuda.current_stream(out.device)
    _check(load_library().lbm_seeded_density(nx, ny, nz, seed, rho_mean, noise_amp,
                                             ctypes.c_void_p(out.data_ptr()),
                                             ctypes.c_void_p(s.cuda_stream)))
    return out


def lbm_structure_functions(h: _Handle, k0: int, k1: int, q: int, r_max: int):
    """(S2[r_max], S4[r_max]) for r = 1..r_max, horizontal increments over planes k0..k1-1."""
    import torch
    lib = load_library()
    nbytes = lib.lbm_structure_work_bytes(h.h, k0, k1, r_max)
    if nbytes == 0:
        raise LbmError(-1, "invalid planes or r_max")
    work = torch.empty(nbytes // 8, dtype=torch.float64, device=h.workspace.device)
    out = (ctypes.c_double * (2 * r_max))()
    _check(lib.lbm_structure_functions(h.h, k0, k1, q, r_max, ctypes.c_void_p(work.data_ptr()),
                                       nbytes, out))
    a = np.array(out[:])
    return a[:r_max], a[r_max:]


def lbm_get_state(h: _Handle, out=None):
    """Canonical FP64 state (38, nz, ny, nx) as a cuda tensor."""
    import torch
    if out is None:
        out = torch.empty((38, h.p.nz, h.p.ny, h.p.nx), dtype=torch.float64,
                          device=h.workspace.device)
    _check(load_library().lbm_get_state(h.h, _dev_ptr(out, torch.float64, 38 * h.p.n)))
    return out


def lbm_set_state(h: _Handle, state):
    import torch
    _check(load_library().lbm_set_state(h.h, _dev_ptr(state, torch.float64, 38 * h.p.n)))


def lbm_adjoint_step(h: _Handle, state, adj_in, adj_out, grads=None):
    """adj_out = (ds_{t+1}/ds_t)^T adj_in; grads (numpy float64[2]) += [dJ/dG, dJ/dT_d]."""
    import torch
    n = 38 * h.p.n
    g = (ctypes.c_double * 2)(*(grads if grads is not None else [0.0, 0.0]))
    _check(load_library().lbm_adjoint_step(h.h, _dev_ptr(state, torch.float64, n),
                                           _dev_ptr(adj_in, torch.float64, n),
                                           _dev_ptr(adj_out, torch.float64, n), g))
    if grads is not None:
        grads[0], grads[1] = g[0], g[1]
    return adj_out


def lbm_adjoint_qbot(h: _Handle, state, weight=0.0, adj=None, grads=None) -> float:
    """q_bot of the state; adj += weight * dq/dstate; grads[1] += weight * dq/dT_d."""
    import torch
    n = 38 * h.p.n
    q = ctypes.c_double()
    g = (ctypes.c_double * 2)(*(grads if grads is not None else [0.0, 0.0]))
    ap = _dev_ptr(adj, torch.float64, n) if adj is not None else None
    _check(load_library().lbm_adjoint_qbot(h.h, _dev_ptr(state, torch.float64, n),
                                           float(weight), ap, ctypes.byref(q), g))
    if grads is not None:
        grads[0], grads[1] = g[0], g[1]
    return q.value


def lbm_adjoint_init_rho(h: _Handle, adj0, T0=None, out=None):
    import torch
    if out is None:
        out = torch.empty(h.p.n, dtype=torch.float64, device=adj0.device)
    T0p = _dev_ptr(T0, torch.float64, h.p.n) if T0 is not None else None
    _check(load_library().lbm_adjoint_init_rho(h.h, _dev_ptr(adj0, torch.float64, 38 * h.p.n),
                                               T0p, _dev_ptr(out, torch.float64, h.p.n)))
    return out


def lbm_pressure_work(h: _Handle) -> np.ndarray:
    """<P d_j v_j>(k), nz doubles (eq. (heat2), eq. (flux))."""
    import torch
    work = torch.empty(5 * h.p.n, dtype=torch.float64, device=h.workspace.device)
    out = (ctypes.c_double * h.p.nz)()
    _check(load_library().lbm_pressure_work(h.h, ctypes.c_void_p(work.data_ptr()),
                                            5 * h.p.n * 8, out))
    return np.array(out[:])


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _raw_ptr(t):
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous cuda tensor")
    return ctypes.c_void_p(t.data_ptr())


def lbm_stream_copy(src, dst, nbytes: int, nontemporal: bool = False, stream=None):
    """Plain device copy of nbytes (bandwidth reference; asynchronous)."""
    if src.numel() * src.element_size() < nbytes or dst.numel() * dst.element_size() < nbytes:
        raise ValueError("buffers smaller than nbytes")
    _check(load_library().lbm_stream_copy(_raw_ptr(src), _raw_ptr(dst), int(nbytes),
                                          1 if nontemporal else 0, _stream_ptr(stream)))


def lbm_stream_rows(src, dst, rows: int, row_stride: int, row_bytes: int, stream=None):
    """The step's row-streaming pattern without arithmetic (bandwidth
    reference; asynchronous)."""
    need = rows * row_stride
    if src.numel() * src.element_size() < need or dst.numel() * dst.element_size() < need:
        raise ValueError("buffers smaller than rows * row_stride")
    _check(load_library().lbm_stream_rows(_raw_ptr(src), _raw_ptr(dst), int(rows), int(row_stride),
                                          int(row_bytes), _stream_ptr(stream)))


def lbm_destroy(h: _Handle):
    if h.h:
        load_library().lbm_destroy(h.h)
        h.h = None


class Lattice:
    """Convenience wrapper: Lattice(params, rho0).step(n).moments() ..."""

    def __init__(self, p: Params, rho0, T0=None, stream=None):
        import torch
        rho0 = torch.as_tensor(rho0, dtype=torch.float64)
        if not rho0.is_cuda:
            rho0 = rho0.cuda()
        rho0 = rho0.contiguous().reshape(-1)
        if T0 is not None:
            T0 = torch.as_tensor(T0, dtype=torch.float64).cuda().contiguous().reshape(-1)
        self.p = p
        self.h = lbm_init(p, rho0, T0, stream)

    def step(self, n: int = 1):
        lbm_step(self.h, n)
        return self

    def set_check(self, every: int, mass_tol: float = 1e-6):
        """Numeric guard: lbm_step checks the state every `every` steps."""
        _check(load_library().lbm_set_check(self.h.h, int(every), float(mass_tol)))
        return self

    @property
    def t(self) -> int:
        return lbm_time(self.h)

    def moments(self, fields=None):
        return lbm_moments(self.h, fields)

    def fields(self):
        import torch
        out = torch.empty(5 * self.p.n, dtype=torch.float64, device=self.h.workspace.device)
        tot = lbm_moments(self.h, out)
        return tot, out.view(5, self.p.nz, self.p.ny, self.p.nx)

    def nusselt(self):
        return lbm_nusselt(self.h)

    def pressure_work(self):
        return lbm_pressure_work(self.h)

    def histogram(self, k0, k1, qx, x_range, nx_bins, qy=-1, y_range=(0.0, 1.0), ny_bins=1):
        return lbm_histogram(self.h, k0, k1, qx, x_range, nx_bins, qy, y_range, ny_bins)

    def structure_functions(self, k0, k1, q, r_max):
        return lbm_structure_functions(self.h, k0, k1, q, r_max)

    def state(self):
        return lbm_get_state(self.h)

    def set_state(self, s):
        import torch
        lbm_set_state(self.h, torch.as_tensor(s, dtype=torch.float64).cuda().contiguous())
        return self
