"""Thin ctypes binding of the C ABI in include/sipg.h.

Argument marshalling only: every step of the operator runs in the HIP
library libsipg.so.  PyTorch provides device memory and streams.  If the
library has not been built, importing this module raises ImportError (there
is no fallback path).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsipg.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with paper_1907_08492_amd/build.py")
# PyTorch ships its own HIP runtime.  Load it first so that libsipg.so binds
# to that same runtime (one HIP runtime per process; torch allocates the
# buffers and streams the library works on).
try:
    import torch as _torch_first  # noqa: F401
except ImportError:  # host-only use (tables, launch shapes) without torch
    _torch_first = None
lib = C.CDLL(LIB_PATH)

# ----------------------------------------------------------------- constants
SIPG_OK, SIPG_E_ARG, SIPG_E_OOM, SIPG_E_HIP, SIPG_E_UNSUPPORTED = 0, -1, -2, -3, -4
SIPG_E_NOTREADY, SIPG_E_NOCONV, SIPG_E_BUDGET = -5, -6, -7
BASIS = {"hermite_like": 0, "nodal_gl": 1, "nodal_gauss": 2}
DTYPE = {"f64": 0, "f32": 1}
GEOMETRY = {"auto": 0, "cell": 1, "qpoint": 2}
BC_MODES = {"T": 0, "TT": 1, "VALUES": 2, "PJACOBI": 3, "FDM": 4}
SMOOTHERS = {"pjacobi": 0, "fdm": 1}

EXPORTED = [
    "sipg_setup", "sipg_destroy", "sipg_ndofs", "sipg_get_info", "sipg_apply", "sipg_apply_pjacobi",
    "sipg_basis_change", "sipg_compute_gl_diagonal", "sipg_cg_solve",
    "sipg_last_error", "sipg_host_tables", "sipg_launch_shape",
    "sipg_mg_default_opts", "sipg_mg_setup", "sipg_mg_destroy", "sipg_mg_get_info",
    "sipg_mg_apply_vcycle", "sipg_mg_solve", "sipg_mg_solve_many", "sipg_mg_transfer", "sipg_mg_level_ndofs",
    "sipg_assemble_rhs_sines",
    "sipg_server_default_opts", "sipg_server_create", "sipg_submit", "sipg_poll", "sipg_wait",
    "sipg_release", "sipg_server_stats", "sipg_server_destroy", "sipg_copy_device",
    "sipg_batch_create", "sipg_batch_apply", "sipg_batch_get_info", "sipg_batch_destroy",
    "sipg_host_fdm_tables", "sipg_mg_level_degree", "sipg_batch_tune",
    "sipg_cg_solve_static", "sipg_cg_static_max_dofs", "sipg_host_block_order", "sipg_stream_bound",
    "sipg_setup_slab", "sipg_ghost_size", "sipg_pack_ghost", "sipg_apply_slab",
]


class SipgMesh(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("lo", C.c_double * 3), ("hi", C.c_double * 3),
                ("lin", C.c_double * 9), ("deform_amp", C.c_double), ("width", C.c_double * 3)]


class SipgOpInfo(C.Structure):
    _fields_ = [("degree", C.c_int32), ("basis", C.c_int32), ("dtype", C.c_int32),
                ("geometry", C.c_int32), ("n", C.c_int32 * 3), ("ndofs", C.c_int64),
                ("device_bytes", C.c_int64), ("cells_per_block", C.c_int32),
                ("threads_per_block", C.c_int32), ("diagonal_metric", C.c_int32)]


class SipgSolveInfo(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("initial_residual", C.c_double),
                ("final_residual", C.c_double), ("true_residual", C.c_double)]


class SipgMgOpts(C.Structure):
    _fields_ = [("smoother_degree", C.c_int32), ("lanczos_steps", C.c_int32), ("range_lo", C.c_double),
                ("range_hi", C.c_double), ("coarse_reduction", C.c_double), ("min_coarse_cells", C.c_int32),
                ("precision", C.c_int32), ("smoother", C.c_int32), ("p_coarsening", C.c_int32),
                ("fused_smoother", C.c_int32), ("lanczos_start", C.c_int32), ("graded_coarsening", C.c_int32),
                ("coarse_direct_max_dofs", C.c_int32)]


class SipgMgInfo(C.Structure):
    _fields_ = [("levels", C.c_int32), ("ndofs", C.c_int64), ("precision", C.c_int32),
                ("lambda_max_fine", C.c_double), ("lambda_min_coarse", C.c_double),
                ("lambda_max_coarse", C.c_double), ("coarse_steps", C.c_int32), ("device_bytes", C.c_int64)]


class SipgServerOpts(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_int64), ("workers", C.c_int32), ("precision", C.c_int32),
                ("smoother", C.c_int32), ("p_coarsening", C.c_int32), ("coarse_reduction", C.c_double),
                ("graded_coarsening", C.c_int32), ("coarse_direct_max_dofs", C.c_int32),
                ("batch_max_rhs", C.c_int32), ("batch_max_dofs", C.c_int64)]


class SipgRequest(C.Structure):
    _fields_ = [("mesh", SipgMesh), ("degree", C.c_int32), ("penalty_factor", C.c_double),
                ("basis", C.c_int32), ("nmodes", C.c_int32), ("amps", C.c_double * 16),
                ("waves", (C.c_int32 * 3) * 16), ("rel_tol", C.c_double), ("max_iter", C.c_int32),
                ("x_out", C.c_void_p)]


class SipgResult(C.Structure):
    _fields_ = [("status", C.c_int32), ("iterations", C.c_int32), ("true_residual", C.c_double),
                ("rel_residual", C.c_double), ("queue_s", C.c_double), ("solve_s", C.c_double),
                ("total_s", C.c_double), ("ndofs", C.c_int64), ("x", C.c_void_p)]


class SipgServerStats(C.Structure):
    _fields_ = [("queued", C.c_int64), ("completed", C.c_int64), ("cached_hierarchies", C.c_int64),
                ("used_bytes", C.c_int64), ("peak_bytes", C.c_int64), ("batched_solves", C.c_int64),
                ("batched_requests", C.c_int64)]


class SipgBatchInfo(C.Structure):
    _fields_ = [("nops", C.c_int32), ("launches", C.c_int32), ("ndofs", C.c_int64),
                ("ncells", C.c_int64), ("workgroups", C.c_int64), ("device_bytes", C.c_int64),
                ("per_operator_groups", C.c_int32), ("streams", C.c_int32)]


_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class SipgAllocator(C.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("ctx", C.c_void_p)]


class SipgTables1D(C.Structure):
    _fields_ = [(name, C.POINTER(C.c_double)) for name in (
        "points", "weights", "shape", "shape_grad", "colloc_grad", "face_value0",
        "face_grad0", "face_value1", "face_grad1", "to_gl")]


_vp = C.c_void_p
lib.sipg_setup.argtypes = [C.POINTER(SipgMesh), C.c_int, C.c_double, C.c_int, C.c_int, C.c_int,
                           C.POINTER(SipgAllocator), _vp, C.POINTER(_vp)]
lib.sipg_destroy.argtypes = [_vp]
lib.sipg_ndofs.argtypes = [_vp]
lib.sipg_ndofs.restype = C.c_int64
lib.sipg_get_info.argtypes = [_vp, C.POINTER(SipgOpInfo)]
lib.sipg_apply.argtypes = [_vp, _vp, _vp, _vp]
lib.sipg_apply_pjacobi.argtypes = [_vp, _vp, _vp, _vp, _vp]
lib.sipg_basis_change.argtypes = [_vp, C.c_int, _vp, _vp, _vp]
lib.sipg_stream_bound.argtypes = [_vp, _vp, _vp, _vp, _vp]
lib.sipg_setup_slab.argtypes = [C.POINTER(SipgMesh), C.c_int, C.c_int, C.c_int, C.c_double, C.c_int, C.c_int,
                                C.c_int, C.POINTER(SipgAllocator), _vp, C.POINTER(_vp)]
lib.sipg_ghost_size.argtypes = [_vp]
lib.sipg_ghost_size.restype = C.c_int64
lib.sipg_pack_ghost.argtypes = [_vp, C.c_int, _vp, _vp, _vp]
lib.sipg_apply_slab.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp]
lib.sipg_compute_gl_diagonal.argtypes = [_vp, _vp, _vp]
lib.sipg_cg_solve.argtypes = [_vp, _vp, _vp, C.c_double, C.c_int, C.POINTER(SipgSolveInfo), _vp]
lib.sipg_cg_solve_static.argtypes = [_vp, _vp, _vp, C.c_double, C.c_int, C.POINTER(SipgSolveInfo), _vp]
lib.sipg_host_block_order.argtypes = [C.c_int, C.c_int, C.POINTER(C.c_int32)]
lib.sipg_cg_static_max_dofs.argtypes = []
lib.sipg_cg_static_max_dofs.restype = C.c_int64
lib.sipg_last_error.restype = C.c_char_p
lib.sipg_host_tables.argtypes = [C.c_int, C.c_int, C.POINTER(SipgTables1D)]
lib.sipg_launch_shape.argtypes = [C.c_int, C.c_int, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                  C.POINTER(C.c_int64)]
lib.sipg_mg_default_opts.argtypes = [C.POINTER(SipgMgOpts)]
lib.sipg_mg_setup.argtypes = [C.POINTER(SipgMesh), C.c_int, C.c_double, C.c_int, C.POINTER(SipgMgOpts),
                              C.POINTER(SipgAllocator), _vp, C.POINTER(_vp)]
lib.sipg_mg_destroy.argtypes = [_vp]
lib.sipg_mg_get_info.argtypes = [_vp, C.POINTER(SipgMgInfo)]
lib.sipg_mg_apply_vcycle.argtypes = [_vp, _vp, _vp, _vp]
lib.sipg_mg_solve.argtypes = [_vp, _vp, _vp, C.c_double, C.c_int, C.POINTER(SipgSolveInfo), _vp]
lib.sipg_mg_solve_many.argtypes = [_vp, C.c_int, _vp, _vp, C.c_double, C.c_int, C.POINTER(SipgSolveInfo), _vp]
lib.sipg_mg_transfer.argtypes = [_vp, C.c_int, C.c_int, _vp, _vp, _vp]
lib.sipg_mg_level_ndofs.argtypes = [_vp, C.c_int, C.POINTER(C.c_int64), C.POINTER(C.c_int32)]
lib.sipg_mg_level_degree.argtypes = [_vp, C.c_int, C.POINTER(C.c_int32)]
lib.sipg_assemble_rhs_sines.argtypes = [_vp, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_int), _vp, _vp]
lib.sipg_server_default_opts.argtypes = [C.POINTER(SipgServerOpts)]
lib.sipg_server_create.argtypes = [C.POINTER(SipgServerOpts), C.POINTER(SipgAllocator), C.POINTER(_vp)]
lib.sipg_submit.argtypes = [_vp, C.POINTER(SipgRequest), C.POINTER(C.c_uint64)]
lib.sipg_poll.argtypes = [_vp, C.c_uint64, C.POINTER(SipgResult)]
lib.sipg_wait.argtypes = [_vp, C.c_uint64, C.POINTER(SipgResult)]
lib.sipg_release.argtypes = [_vp, C.c_uint64, _vp]
lib.sipg_server_stats.argtypes = [_vp, C.POINTER(SipgServerStats)]
lib.sipg_server_destroy.argtypes = [_vp]
lib.sipg_copy_device.argtypes = [_vp, _vp, C.c_size_t, _vp]
lib.sipg_batch_create.argtypes = [C.c_int, C.POINTER(_vp), C.POINTER(_vp), C.POINTER(_vp), C.POINTER(_vp)]
lib.sipg_batch_apply.argtypes = [_vp, _vp]
lib.sipg_batch_get_info.argtypes = [_vp, C.POINTER(SipgBatchInfo)]
lib.sipg_batch_destroy.argtypes = [_vp]
lib.sipg_batch_tune.argtypes = [_vp, C.c_int, _vp]
lib.sipg_host_fdm_tables.argtypes = [C.c_int, C.c_int, C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_double)]
for _f in EXPORTED:
    if _f not in ("sipg_ndofs", "sipg_last_error", "sipg_cg_static_max_dofs", "sipg_ghost_size"):
        getattr(lib, _f).restype = C.c_int


class SipgError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where} failed ({code}): {lib.sipg_last_error().decode()}")


def _check(code: int, where: str):
    if code != SIPG_OK:
        raise SipgError(code, where)


# ------------------------------------------------------------------ host-only
def host_tables(degree: int, basis: str = "hermite_like") -> dict:
    """1D tables computed by the library's host code (no GPU needed)."""
    n = degree + 1
    arrays = {k: np.zeros(n * n if k in ("shape", "shape_grad", "colloc_grad", "to_gl") else n)
              for k, _ in SipgTables1D._fields_}
    t = SipgTables1D(**{k: v.ctypes.data_as(C.POINTER(C.c_double)) for k, v in arrays.items()})
    _check(lib.sipg_host_tables(degree, BASIS[basis], C.byref(t)), "sipg_host_tables")
    for k in ("shape", "shape_grad", "colloc_grad", "to_gl"):
        arrays[k] = arrays[k].reshape(n, n)
    return arrays


def host_fdm_tables(degree: int, basis: str = "hermite_like", penalty: float = 2.0):
    """(Z^T, lambda) of the block preconditioner, from the library's host code."""
    n = degree + 1
    zt = np.zeros(n * n)
    lam = np.zeros(n)
    _check(lib.sipg_host_fdm_tables(degree, BASIS[basis], float(penalty),
                                    zt.ctypes.data_as(C.POINTER(C.c_double)),
                                    lam.ctypes.data_as(C.POINTER(C.c_double))), "sipg_host_fdm_tables")
    return zt.reshape(n, n), lam


def launch_shape(degree: int, dtype: str = "f64"):
    """(cells per workgroup, threads per workgroup, dynamic LDS bytes)."""
    cpb, nt, lds = C.c_int32(), C.c_int32(), C.c_int64()
    _check(lib.sipg_launch_shape(degree, DTYPE[dtype], C.byref(cpb), C.byref(nt), C.byref(lds)),
           "sipg_launch_shape")
    return cpb.value, nt.value, lds.value


def host_block_order(nblocks: int, layer_blocks: int) -> np.ndarray:
    """Block visited by each workgroup of the single-operator product kernel."""
    out = np.zeros(nblocks, dtype=np.int32)
    _check(lib.sipg_host_block_order(int(nblocks), int(layer_blocks), out.ctypes.data_as(C.POINTER(C.c_int32))),
           "sipg_host_block_order")
    return out


def make_mesh(mesh) -> SipgMesh:
    """Convert any object with n, lo, hi, lin, deform_amp (and optionally
    width, for a graded brick) attributes."""
    m = SipgMesh()
    for d in range(3):
        m.n[d] = int(mesh.n[d])
        m.lo[d] = float(mesh.lo[d])
        m.hi[d] = float(mesh.hi[d])
    lin = getattr(mesh, "lin", None)
    if lin is not None:
        flat = np.asarray(lin, dtype=np.float64).reshape(9)
        for i in range(9):
            m.lin[i] = float(flat[i])
    m.deform_amp = float(getattr(mesh, "deform_amp", 0.0))
    width = getattr(mesh, "width", None)
    if width is not None:
        for d in range(3):
            m.width[d] = float(width[d])
    return m


# --------------------------------------------------------------- device side
def _torch():
    import torch  # noqa: WPS433 (imported lazily: host-only users need no torch)
    return torch


def _stream_ptr(stream) -> int:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


# PyTorch's caching allocator as the library's device memory provider: the
# operator, solver and request-loop memory then comes from (and goes back to)
# torch's pool.  The callbacks run on the calling thread (the request loop's
# workers too); blocks are taken on the current device.  The library returns a
# block only once its own queued work on it is finished.
@_ALLOC_FN
def _torch_alloc(nbytes, ctx):
    try:
        torch = _torch()
        return torch.cuda.caching_allocator_alloc(int(nbytes), device=torch.cuda.current_device())
    except Exception:
        return None


@_FREE_FN
def _torch_free(ptr, ctx):
    _torch().cuda.caching_allocator_delete(int(ptr))


TORCH_ALLOCATOR = SipgAllocator(_torch_alloc, _torch_free, None)


def _allocator(kind):
    """C pointer for allocator="torch" (PyTorch's caching allocator) or None
    (hipMalloc inside the library)."""
    if kind is None:
        return None
    if kind == "torch":
        return C.byref(TORCH_ALLOCATOR)
    raise ValueError("allocator must be 'torch' or None")


@dataclass
class SolveInfo:
    iterations: int
    initial_residual: float
    final_residual: float
    true_residual: float
    status: int


class Operator:
    """The SIPG operator of one mesh, degree and basis on the current device."""

    def __init__(self, mesh, degree: int, penalty: float = 2.0, basis: str = "hermite_like",
                 dtype: str = "f64", geometry: str = "auto", stream=None, allocator="torch", slab=None):
        """slab=(z0, z1): the operator of the cells z0 <= iz < z1 of the mesh
        (one GPU's share of a z-partition, sipg_setup_slab)."""
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("Operator needs a GPU (HIP device)")
        self._allocator = allocator
        self.degree = int(degree)
        self.basis = basis
        self.dtype_name = dtype
        self.torch_dtype = torch.float64 if dtype == "f64" else torch.float32
        self._mesh = make_mesh(mesh)
        h = _vp()
        if slab is None:
            _check(lib.sipg_setup(C.byref(self._mesh), self.degree, float(penalty), BASIS[basis],
                                  DTYPE[dtype], GEOMETRY[geometry], _allocator(allocator), _vp(_stream_ptr(stream)),
                                  C.byref(h)), "sipg_setup")
        else:
            _check(lib.sipg_setup_slab(C.byref(self._mesh), int(slab[0]), int(slab[1]), self.degree, float(penalty),
                                       BASIS[basis], DTYPE[dtype], GEOMETRY[geometry], _allocator(allocator),
                                       _vp(_stream_ptr(stream)), C.byref(h)), "sipg_setup_slab")
        self.slab = None if slab is None else (int(slab[0]), int(slab[1]))
        self._h = h
        self.ndofs = int(lib.sipg_ndofs(h))
        info = SipgOpInfo()
        _check(lib.sipg_get_info(h, C.byref(info)), "sipg_get_info")
        self.info = info

    @property
    def handle(self):
        return self._h

    def _vec(self, t, name):
        torch = _torch()
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise TypeError(f"{name} must be a CUDA/HIP tensor")
        if t.dtype != self.torch_dtype or t.numel() != self.ndofs or not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous {self.torch_dtype} with {self.ndofs} elements")
        return _vp(t.data_ptr())

    def empty(self):
        return _torch().empty(self.ndofs, dtype=self.torch_dtype, device="cuda")

    def ghost_size(self) -> int:
        return int(lib.sipg_ghost_size(self._h))

    def pack_ghost(self, side: int, x, out=None, stream=None):
        """The layers of the bottom (side 0) or top (side 1) cell row that the
        neighbouring slab reads (sipg_pack_ghost)."""
        torch = _torch()
        g = torch.empty(self.ghost_size(), dtype=self.torch_dtype, device="cuda") if out is None else out
        if g.dtype != self.torch_dtype or g.numel() != self.ghost_size() or not g.is_contiguous():
            raise ValueError(f"out must be contiguous {self.torch_dtype} with {self.ghost_size()} elements")
        _check(lib.sipg_pack_ghost(self._h, int(side), self._vec(x, "x"), _vp(g.data_ptr()), _vp(_stream_ptr(stream))),
               "sipg_pack_ghost")
        return g

    def apply_slab(self, x, ghost_lo=None, ghost_hi=None, y=None, z=None, stream=None):
        """y = A x on a slab with the neighbours' ghost layers; with z, also
        z = P^-1 y (sipg_apply_slab).  Returns y (and z when given)."""
        y = self.empty() if y is None else y
        gp = lambda g: None if g is None else _vp(g.data_ptr())
        _check(lib.sipg_apply_slab(self._h, self._vec(x, "x"), gp(ghost_lo), gp(ghost_hi), self._vec(y, "y"),
                                   None if z is None else self._vec(z, "z"), _vp(_stream_ptr(stream))),
               "sipg_apply_slab")
        return y if z is None else (y, z)

    def apply(self, x, out=None, stream=None):
        """out = A x (stream ordered)."""
        y = self.empty() if out is None else out
        _check(lib.sipg_apply(self._h, self._vec(x, "x"), self._vec(y, "out"), _vp(_stream_ptr(stream))),
               "sipg_apply")
        return y

    def apply_pjacobi(self, x, y=None, z=None, stream=None):
        """y = A x and z = P^-1 y (eq. (jacobi)) in one pass; needs
        compute_gl_diagonal first.  Returns (y, z)."""
        y = self.empty() if y is None else y
        z = self.empty() if z is None else z
        _check(lib.sipg_apply_pjacobi(self._h, self._vec(x, "x"), self._vec(y, "y"), self._vec(z, "z"),
                                      _vp(_stream_ptr(stream))), "sipg_apply_pjacobi")
        return y, z

    def stream_bound(self, x, y, z, stream=None):
        """The step's bytes moved with no arithmetic (sipg_stream_bound): a
        measurement of the HBM bound of apply_pjacobi; y, z get meaningless
        values."""
        _check(lib.sipg_stream_bound(self._h, self._vec(x, "x"), self._vec(y, "y"), self._vec(z, "z"),
                                     _vp(_stream_ptr(stream))), "sipg_stream_bound")

    def basis_change(self, mode: str, x, out=None, stream=None):
        y = self.empty() if out is None else out
        _check(lib.sipg_basis_change(self._h, BC_MODES[mode], self._vec(x, "in"), self._vec(y, "out"),
                                     _vp(_stream_ptr(stream))), "sipg_basis_change")
        return y

    def compute_gl_diagonal(self, return_diag: bool = True, stream=None):
        d = self.empty() if return_diag else None
        _check(lib.sipg_compute_gl_diagonal(self._h, self._vec(d, "diag") if d is not None else None,
                                            _vp(_stream_ptr(stream))), "sipg_compute_gl_diagonal")
        return d

    def cg_solve(self, b, x=None, rel_tol: float = 1e-10, max_iter: int = 10000, stream=None,
                 raise_on_noconv: bool = True):
        torch = _torch()
        if self.dtype_name != "f64":
            raise ValueError("cg_solve needs an f64 operator")
        if x is None:
            x = torch.zeros_like(b)
        info = SipgSolveInfo()
        rc = lib.sipg_cg_solve(self._h, self._vec(b, "b"), self._vec(x, "x"), float(rel_tol), int(max_iter),
                               C.byref(info), _vp(_stream_ptr(stream)))
        if rc != SIPG_OK and (rc != SIPG_E_NOCONV or raise_on_noconv):
            raise SipgError(rc, "sipg_cg_solve")
        return x, SolveInfo(info.iterations, info.initial_residual, info.final_residual,
                            info.true_residual, rc)

    def cg_solve_static(self, b, x, rel_tol: float = 1e-10, max_iter: int = 10000, stream=None,
                        raise_on_noconv: bool = True):
        """cg_solve with the library's fixed work arrays (sipg_cg_solve_static):
        no device allocation at all, x provided by the caller."""
        if self.dtype_name != "f64":
            raise ValueError("cg_solve_static needs an f64 operator")
        info = SipgSolveInfo()
        rc = lib.sipg_cg_solve_static(self._h, self._vec(b, "b"), self._vec(x, "x"), float(rel_tol),
                                      int(max_iter), C.byref(info), _vp(_stream_ptr(stream)))
        if rc != SIPG_OK and (rc != SIPG_E_NOCONV or raise_on_noconv):
            raise SipgError(rc, "sipg_cg_solve_static")
        return x, SolveInfo(info.iterations, info.initial_residual, info.final_residual,
                            info.true_residual, rc)

    def assemble_rhs(self, amps, waves, out=None, stream=None):
        """b for f = sum_m amps[m] sin(w0 pi x) sin(w1 pi y) sin(w2 pi z)."""
        amps = np.ascontiguousarray(amps, dtype=np.float64).reshape(-1)
        waves = np.ascontiguousarray(waves, dtype=np.int32).reshape(-1, 3)
        b = self.empty() if out is None else out
        _check(lib.sipg_assemble_rhs_sines(self._h, len(amps), amps.ctypes.data_as(C.POINTER(C.c_double)),
                                           waves.ctypes.data_as(C.POINTER(C.c_int)), self._vec(b, "out"),
                                           _vp(_stream_ptr(stream))), "sipg_assemble_rhs_sines")
        return b

    def close(self):
        if getattr(self, "_h", None):
            if self._allocator == "torch":
                # hipFree would wait for the device; the caching allocator does
                # not, so queued work on the operator's memory ends first
                _torch().cuda.synchronize()
            lib.sipg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """y_i = A_i x_i for many operators at once (sipg_batch_*).  The vectors
    are bound at construction; the batch keeps references to the operators
    and tensors so that they outlive it."""

    def __init__(self, ops, xs, ys):
        if not (len(ops) == len(xs) == len(ys)) or len(ops) == 0:
            raise ValueError("ops, xs and ys must be non-empty lists of equal length")
        n = len(ops)
        hops = (_vp * n)(*[op.handle for op in ops])
        hx = (_vp * n)(*[op._vec(x, f"xs[{i}]") for i, (op, x) in enumerate(zip(ops, xs))])
        hy = (_vp * n)(*[op._vec(y, f"ys[{i}]") for i, (op, y) in enumerate(zip(ops, ys))])
        h = _vp()
        _check(lib.sipg_batch_create(n, hops, hx, hy, C.byref(h)), "sipg_batch_create")
        self._h = h
        self._keep = (list(ops), list(xs), list(ys))
        info = SipgBatchInfo()
        _check(lib.sipg_batch_get_info(h, C.byref(info)), "sipg_batch_get_info")
        self.info = info

    def apply(self, stream=None):
        _check(lib.sipg_batch_apply(self._h, _vp(_stream_ptr(stream))), "sipg_batch_apply")

    def tune(self, reps: int = 3, stream=None):
        """Pick one grid or one launch per operator for every group by timing."""
        _check(lib.sipg_batch_tune(self._h, int(reps), _vp(_stream_ptr(stream))), "sipg_batch_tune")
        info = SipgBatchInfo()
        _check(lib.sipg_batch_get_info(self._h, C.byref(info)), "sipg_batch_get_info")
        self.info = info

    def close(self):
        if getattr(self, "_h", None):
            lib.sipg_batch_destroy(self._h)
            self._h = None
            self._keep = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Multigrid:
    """FP64 CG preconditioned by a V-cycle (FP32 for precision="mixed")."""

    def __init__(self, mesh, degree: int, penalty: float = 2.0, basis: str = "hermite_like",
                 precision: str = "mixed", stream=None, allocator="torch", **opts):
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("Multigrid needs a GPU (HIP device)")
        self._allocator = allocator
        o = SipgMgOpts()
        _check(lib.sipg_mg_default_opts(C.byref(o)), "sipg_mg_default_opts")
        o.precision = {"mixed": 0, "f64": 1}[precision]
        for k, v in opts.items():
            setattr(o, k, SMOOTHERS[v] if k == "smoother" and isinstance(v, str) else v)
        self._mesh = make_mesh(mesh)
        h = _vp()
        _check(lib.sipg_mg_setup(C.byref(self._mesh), int(degree), float(penalty), BASIS[basis], C.byref(o),
                                 _allocator(allocator), _vp(_stream_ptr(stream)), C.byref(h)), "sipg_mg_setup")
        self._h = h
        self.precision = precision
        info = SipgMgInfo()
        _check(lib.sipg_mg_get_info(h, C.byref(info)), "sipg_mg_get_info")
        self.info = info
        self.ndofs = int(info.ndofs)

    def _vec(self, t, name, dtype=None):
        torch = _torch()
        dtype = torch.float64 if dtype is None else dtype
        if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
            raise TypeError(f"{name} must be a contiguous CUDA/HIP tensor of {dtype}")
        return _vp(t.data_ptr())

    def level(self, level: int):
        n = C.c_int64()
        cells = (C.c_int32 * 3)()
        _check(lib.sipg_mg_level_ndofs(self._h, level, C.byref(n), cells), "sipg_mg_level_ndofs")
        return int(n.value), tuple(cells)

    def level_degree(self, level: int) -> int:
        d = C.c_int32()
        _check(lib.sipg_mg_level_degree(self._h, level, C.byref(d)), "sipg_mg_level_degree")
        return int(d.value)

    def transfer(self, level: int, mode: str, x, out, stream=None):
        dt = _torch().float32 if self.precision == "mixed" else _torch().float64
        _check(lib.sipg_mg_transfer(self._h, level, {"prolongate": 0, "restrict": 1}[mode],
                                    self._vec(x, "in", dt), self._vec(out, "out", dt), _vp(_stream_ptr(stream))),
               "sipg_mg_transfer")
        return out

    def vcycle(self, r, out=None, stream=None):
        z = _torch().empty_like(r) if out is None else out
        _check(lib.sipg_mg_apply_vcycle(self._h, self._vec(r, "r"), self._vec(z, "z"), _vp(_stream_ptr(stream))),
               "sipg_mg_apply_vcycle")
        return z

    def solve(self, b, x=None, rel_tol: float = 1e-10, max_iter: int = 200, stream=None,
              raise_on_noconv: bool = True):
        if x is None:
            x = _torch().zeros_like(b)
        info = SipgSolveInfo()
        rc = lib.sipg_mg_solve(self._h, self._vec(b, "b"), self._vec(x, "x"), float(rel_tol), int(max_iter),
                               C.byref(info), _vp(_stream_ptr(stream)))
        if rc != SIPG_OK and (rc != SIPG_E_NOCONV or raise_on_noconv):
            raise SipgError(rc, "sipg_mg_solve")
        return x, SolveInfo(info.iterations, info.initial_residual, info.final_residual,
                            info.true_residual, rc)

    def solve_many(self, b, x=None, rel_tol: float = 1e-10, max_iter: int = 200, stream=None,
                   raise_on_noconv: bool = True):
        """Solve for the rows of b (nrhs x ndofs, at most 16) together
        (sipg_mg_solve_many); returns x and one SolveInfo per row."""
        if b.dim() != 2 or b.shape[1] != self.ndofs:
            raise ValueError("b must have shape (nrhs, ndofs)")
        if x is None:
            x = _torch().zeros_like(b)
        nrhs = int(b.shape[0])
        infos = (SipgSolveInfo * max(nrhs, 1))()
        rc = lib.sipg_mg_solve_many(self._h, nrhs, self._vec(b, "b"), self._vec(x, "x"), float(rel_tol),
                                    int(max_iter), infos, _vp(_stream_ptr(stream)))
        if rc != SIPG_OK and (rc != SIPG_E_NOCONV or raise_on_noconv):
            raise SipgError(rc, "sipg_mg_solve_many")
        return x, [SolveInfo(i.iterations, i.initial_residual, i.final_residual, i.true_residual, rc)
                   for i in infos[:nrhs]]

    def close(self):
        if getattr(self, "_h", None):
            if self._allocator == "torch":
                _torch().cuda.synchronize()
            lib.sipg_mg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _result_dict(r: SipgResult) -> dict:
    return {k: getattr(r, k) for k, _ in SipgResult._fields_}


class Server:
    """Continuous-batching request loop of multigrid Poisson solves."""

    def __init__(self, hbm_budget_bytes: int = 64 << 30, workers: int = 8, precision: str = "mixed",
                 smoother: str = "fdm", p_coarsening: int = 1, coarse_reduction: float = 10.0,
                 allocator="torch", graded_coarsening: int = 0, coarse_direct_max_dofs: int = 256,
                 batch_max_rhs: int = 8, batch_max_dofs: int = 1 << 20):
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("Server needs a GPU (HIP device)")
        torch.cuda.init()
        o = SipgServerOpts(int(hbm_budget_bytes), int(workers), {"mixed": 0, "f64": 1}[precision],
                           SMOOTHERS[smoother], int(p_coarsening), float(coarse_reduction),
                           int(graded_coarsening), int(coarse_direct_max_dofs), int(batch_max_rhs),
                           int(batch_max_dofs))
        h = _vp()
        _check(lib.sipg_server_create(C.byref(o), _allocator(allocator), C.byref(h)), "sipg_server_create")
        self._h = h

    @staticmethod
    def make_request(mesh, degree: int, amps, waves, penalty: float = 2.0, basis: str = "hermite_like",
                     rel_tol: float = 1e-8, max_iter: int = 200, x_out=None) -> SipgRequest:
        r = SipgRequest()
        r.mesh = make_mesh(mesh)
        r.degree = int(degree)
        r.penalty_factor = float(penalty)
        r.basis = BASIS[basis]
        amps = list(amps)
        waves = [tuple(w) for w in waves]
        r.nmodes = len(amps)
        for i, (a, w) in enumerate(zip(amps, waves)):
            r.amps[i] = float(a)
            for d in range(3):
                r.waves[i][d] = int(w[d])
        r.rel_tol = float(rel_tol)
        r.max_iter = int(max_iter)
        r.x_out = None if x_out is None else int(x_out.data_ptr())
        return r

    def submit(self, req: SipgRequest) -> int:
        t = C.c_uint64()
        _check(lib.sipg_submit(self._h, C.byref(req), C.byref(t)), "sipg_submit")
        return int(t.value)

    def poll(self, ticket: int):
        r = SipgResult()
        rc = lib.sipg_poll(self._h, ticket, C.byref(r))
        if rc == SIPG_E_NOTREADY:
            return None
        _check(rc, "sipg_poll")
        return _result_dict(r)

    def wait(self, ticket: int) -> dict:
        r = SipgResult()
        _check(lib.sipg_wait(self._h, ticket, C.byref(r)), "sipg_wait")
        return _result_dict(r)

    def solution(self, result: dict, stream=None):
        """Copy of a result's device solution as a torch tensor."""
        torch = _torch()
        out = torch.empty(int(result["ndofs"]), dtype=torch.float64, device="cuda")
        _check(lib.sipg_copy_device(_vp(out.data_ptr()), _vp(result["x"]), C.c_size_t(out.numel() * 8),
                                    _vp(_stream_ptr(stream))), "sipg_copy_device")
        return out

    def release(self, ticket: int, stream=None):
        """Forget a finished request; a server-owned solution is freed once the
        work queued on `stream` (default: the current stream) has finished."""
        _check(lib.sipg_release(self._h, ticket, _vp(_stream_ptr(stream))), "sipg_release")

    def stats(self) -> dict:
        st = SipgServerStats()
        _check(lib.sipg_server_stats(self._h, C.byref(st)), "sipg_server_stats")
        return {k: getattr(st, k) for k, _ in SipgServerStats._fields_}

    def close(self):
        if getattr(self, "_h", None):
            lib.sipg_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

