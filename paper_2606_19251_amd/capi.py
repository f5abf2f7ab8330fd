"""ctypes binding of libamggnn.so: the C entry points under their C names.

Argument marshalling only. Pointers are passed as Python ints (for device memory,
``tensor.data_ptr()``); sizes as ints; host arrays as numpy arrays. Every call raises
``AmggError`` on a negative status. Loading fails loudly when the library is missing:
there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libamggnn.so")

AMGG_OK = 0
AMGG_EINVAL = -1
AMGG_EWORKSPACE = -2
AMGG_EHIP = -3
AMGG_ESTATE = -4
AMGG_ENONFINITE = -5
AMGG_MAXIT, AMGG_DIVERGED, AMGG_STAGNATED, AMGG_BREAKDOWN = 1, 2, 3, 4
AMGG_OUTER_STATIONARY, AMGG_OUTER_IR, AMGG_OUTER_FCG = 0, 1, 2
(AMGG_OP_SPMV, AMGG_OP_RESIDUAL, AMGG_OP_SMOOTH, AMGG_OP_JACOBI, AMGG_OP_RESTRICT, AMGG_OP_PROLONG,
 AMGG_OP_COARSE) = range(7)
AMGG_MAX_LEVELS = 16
AMGG_MAX_COARSE_DENSE = 4096


class AmggError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class amgg_level_view(C.Structure):
    _fields_ = [("n", C.c_int32), ("nnz", C.c_int32), ("n_coarse", C.c_int32), ("p_nnz", C.c_int32),
                ("r_rowptr", C.c_void_p), ("r_col", C.c_void_p), ("r_val", C.c_void_p),
                ("a_val32", C.c_void_p), ("p_val32", C.c_void_p), ("r_val32", C.c_void_p),
                ("q_val", C.c_void_p), ("q_val32", C.c_void_p), ("diag", C.c_void_p),
                ("scale", C.c_void_p), ("coarse_inv", C.c_void_p), ("fused_rows", C.c_int32),
                ("pack_rows", C.c_int32 * 3), ("pack_far", C.c_int64 * 3),
                ("stream_cap", C.c_int32 * 3)]


class amgg_solve_opts(C.Structure):
    _fields_ = [("outer", C.c_int), ("inner_precision", C.c_int), ("nu1", C.c_int), ("nu2", C.c_int),
                ("maxit", C.c_int), ("tol", C.c_double), ("fallback", C.c_int), ("div_factor", C.c_double),
                ("stag_ratio", C.c_double), ("stag_window", C.c_int), ("graphs", C.c_int)]


class amgg_solve_info(C.Structure):
    _fields_ = [("iterations", C.c_int), ("vcycles", C.c_int), ("relres", C.c_double), ("status", C.c_int),
                ("fell_back", C.c_int)]


class amgg_hier_sizes(C.Structure):
    _fields_ = [("nlevels", C.c_int), ("singular", C.c_int), ("n", C.c_int32 * AMGG_MAX_LEVELS),
                ("nnz", C.c_int32 * AMGG_MAX_LEVELS), ("p_ncols", C.c_int32 * AMGG_MAX_LEVELS),
                ("p_nnz", C.c_int32 * AMGG_MAX_LEVELS)]


class amgg_hier_host(C.Structure):
    _fields_ = [(k, C.c_void_p * AMGG_MAX_LEVELS) for k in ("rowptr", "col", "val", "p_rowptr", "p_col", "p_val",
                                                              "cf")]


class amgg_judge_info(C.Structure):
    _fields_ = [("learned_wins", C.c_int), ("iterations", C.c_int * 2), ("status", C.c_int * 2),
                ("log10_relres", C.c_double * 2), ("log10_rate", C.c_double * 2), ("ms_per_iter", C.c_double * 2),
                ("predicted_ms", C.c_double * 2)]


class gcin_graph(C.Structure):
    _fields_ = [("n", C.c_int32), ("nnz", C.c_int32), ("rowptr", C.c_void_p), ("col", C.c_void_p),
                ("val", C.c_void_p)]


GCIN_FP32, GCIN_BF16, GCIN_BF16X3 = 0, 1, 2
GCIN_INFERENCE = 1

_VP = C.c_void_p
_I32 = C.c_int32
_I = C.c_int

# name -> (restype, argtypes)
SIGNATURES = {
    "amgg_rs_setup": (_I, [_VP, _VP, _VP, _I32, C.c_double, _I, _I32, C.POINTER(_VP)]),
    "amgg_rs_info": (_I, [_VP, C.POINTER(_I), C.POINTER(_I)]),
    "amgg_rs_level_size": (_I, [_VP, _I, C.POINTER(_I32), C.POINTER(_I32), C.POINTER(_I32), C.POINTER(_I32)]),
    "amgg_rs_copy_level": (_I, [_VP, _I, _VP, _VP, _VP, _VP, _VP, _VP, _VP]),
    "amgg_rs_free": (None, [_VP]),
    "amgg_rs_begin": (_I, [_VP, _VP, _VP, _I32, C.c_double, _I, _I32, C.POINTER(_VP)]),
    "amgg_rs_coarsen": (_I, [_VP, C.POINTER(_I)]),
    "amgg_rs_galerkin": (_I, [_VP]),
    "amgg_rs_push_level": (_I, [_VP, _I32, _VP, _VP, _VP]),
    "amgg_rs_split": (_I, [_VP, _VP, _VP, C.POINTER(_I)]),
    "amgg_rs_setup_query": (_I, [_VP, _VP, _VP, _I32, C.c_double, _I, _I32, C.POINTER(amgg_hier_sizes)]),
    "amgg_rs_setup_fill": (_I, [_VP, _VP, _VP, _I32, C.c_double, _I, _I32, C.POINTER(amgg_hier_host)]),
    "amgg_get_smoother_values": (_I, [_VP, _I, _VP, _VP]),
    "amgg_rs_push_interp": (_I, [_VP, _I32, _VP, _VP, _VP]),
    "amgg_strength_device": (_I, [_I, _I32, _VP, _VP, _VP, _I32, C.c_double, _VP, _VP, _VP, _VP, _VP]),
    "amgg_interp_device": (_I, [_I, _I32, _VP, _VP, _VP, _I32, _VP, _VP, _VP, _VP, _VP, C.POINTER(_I32),
                                C.POINTER(_VP), C.POINTER(_VP), C.POINTER(_VP), C.POINTER(_I32), _VP]),
    "amgg_galerkin_device": (_I, [_I, _I32, _I32, _VP, _VP, _VP, _I32, _VP, _VP, _VP, _I32, _VP, _VP, _VP,
                                  C.c_int64, C.POINTER(_VP), C.POINTER(_VP), C.POINTER(_VP), C.POINTER(_I32), _VP]),
    "amgg_create": (_I, [C.POINTER(_VP), _I, _I]),
    "amgg_destroy": (_I, [_VP]),
    "amgg_last_error": (C.c_char_p, []),
    "amgg_load_level": (_I, [_VP, _I, _I32, _I32, _VP, _VP, _VP]),
    "amgg_load_prolong": (_I, [_VP, _I, _I32, _I32, _I32, _VP, _VP, _VP]),
    "amgg_workspace_bytes": (_I, [_VP, C.POINTER(C.c_size_t)]),
    "amgg_finalize": (_I, [_VP, _I, _VP, C.c_size_t, _VP]),
    "amgg_level_view_get": (_I, [_VP, _I, C.POINTER(amgg_level_view)]),
    "amgg_set_smoother_coeffs": (_I, [_VP, _I, _I, _VP, _VP]),
    "amgg_set_smoother_coeffs_device": (_I, [_VP, _I, _I, _VP, _VP]),
    "amgg_set_smoother_coeffs_device_form": (_I, [_VP, _I, _I, _VP, _I, _VP]),
    "amgg_set_smoother_jacobi": (_I, [_VP, _I, C.c_double, _VP]),
    "amgg_vcycle": (_I, [_VP, _I, _I, _I, _VP, _VP, _VP]),
    "amgg_level_apply": (_I, [_VP, _I, _I, _I, _VP, _VP, _VP, _VP]),
    "amgg_set_fusion": (_I, [_VP, _I]),
    "amgg_set_packed_columns": (_I, [_VP, _I]),
    "amgg_level_apply_timed": (_I, [_VP, _I, _I, _I, _VP, _VP, _VP, _VP, _VP, _VP]),
    "amgg_solve": (_I, [_VP, C.POINTER(amgg_solve_opts), _VP, _VP, C.POINTER(amgg_solve_info), _VP, _I, _VP]),
    "amgg_judge_smoother": (_I, [_VP, C.POINTER(amgg_solve_opts), _I, _I, _VP, _I, _VP, _VP,
                                 C.POINTER(amgg_judge_info), _VP]),
    "amgg_vcycle_loss_adjoint": (_I, [_VP, _I, _I, _I, _I, _VP, _VP, _VP, _VP, _VP]),
    "amgg_set_level_blocks": (_I, [_VP, _I, _I32, _VP, _VP, _VP]),
    "amgg_set_smoother_coeffs_blocks": (_I, [_VP, _I, _I, _VP, _I32, _VP]),
    "amgg_set_smoother_coeffs_blocks_form": (_I, [_VP, _I, _I, _VP, _I32, _I, _VP]),
    "amgg_vcycle_loss_adjoint_blocks": (_I, [_VP, _I, _I, _I, _I, _VP, _VP, _VP, _VP, _I32, _VP]),
    "amgg_chain_loss_grad": (_I, [C.c_int32, C.c_int32, _VP, _VP, _VP, _VP, _VP]),
    "amgg_validation_metric": (_I, [C.c_int32, _VP, _VP, _VP, _VP]),
    "amgg_cast_scale_f64_f32": (_I, [_VP, _VP, C.c_int64, C.c_double, _VP]),
    "gcin_param_count": (C.c_int64, [_I]),
    "gcin_param_count_hidden": (C.c_int64, [_I, _I]),
    "gcin_batch_workspace_bytes": (_I, [_I, _VP, _VP, C.POINTER(C.c_size_t)]),
    "gcin_batch_workspace_bytes_hidden": (_I, [_I, _I, _VP, _VP, C.POINTER(C.c_size_t)]),
    "gcin_batch_create": (_I, [_I, C.POINTER(gcin_graph), _VP, C.c_size_t, _VP, C.POINTER(_VP)]),
    "gcin_batch_create_hidden": (_I, [_I, _I, C.POINTER(gcin_graph), _VP, C.c_size_t, _VP, C.POINTER(_VP)]),
    "gcin_batch_workspace_bytes_ex": (_I, [_I, _I, _I, _VP, _VP, C.POINTER(C.c_size_t)]),
    "gcin_batch_create_ex": (_I, [_I, _I, _I, C.POINTER(gcin_graph), _VP, C.c_size_t, _VP, C.POINTER(_VP)]),
    "gcin_batch_destroy": (_I, [_VP]),
    "gcin_forward": (_I, [_VP, _I, _I, _VP, _VP, _VP]),
    "gcin_backward": (_I, [_VP, _I, _I, _VP, _VP, _VP, _VP]),
    "gcin_tile_gemm_check": (_I, [_VP, _VP, _VP, _VP, _VP]),
    "adam_scratch_bytes": (C.c_size_t, []),
    "adam_step": (_I, [_VP, _VP, _VP, _VP, C.c_int64, C.c_float, C.c_float, C.c_float, C.c_float, _I, C.c_float,
                       _VP, _VP, _VP]),
    "adam_step_noalloc": (_I, [_VP, _VP, _VP, _VP, C.c_int64, C.c_float, C.c_float, C.c_float, C.c_float, _I,
                               C.c_float, _VP, _VP]),
}

_lib = None


def lib():
    """Load libamggnn.so (once); raises if it has not been built."""
    global _lib
    if _lib is None:
        # The library resolves the HIP runtime by soname; loading torch first (when it is
        # installed) makes the process use one runtime for torch's memory and our kernels.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} not found: build it with `python -m paper_2606_19251_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def amgg_last_error() -> str:
    return lib().amgg_last_error().decode()


def _check(rc: int, name: str) -> int:
    if rc < 0:
        raise AmggError(rc, f"{name}: {amgg_last_error()}")
    return rc


def _np_ptr(a):
    return None if a is None else a.ctypes.data


# ---------------------------------------------------------------------------- host setup
def amgg_rs_setup(rowptr: np.ndarray, col: np.ndarray, val: np.ndarray, n: int, theta: float,
                  max_levels: int, max_coarse: int) -> int:
    rowptr = np.ascontiguousarray(rowptr, np.int32)
    col = np.ascontiguousarray(col, np.int32)
    val = np.ascontiguousarray(val, np.float64)
    h = _VP()
    _check(lib().amgg_rs_setup(_np_ptr(rowptr), _np_ptr(col), _np_ptr(val), n, theta, max_levels, max_coarse,
                               C.byref(h)), "amgg_rs_setup")
    return h.value


def amgg_rs_info(h: int):
    nl, sg = _I(), _I()
    _check(lib().amgg_rs_info(h, C.byref(nl), C.byref(sg)), "amgg_rs_info")
    return nl.value, sg.value


def amgg_rs_level_size(h: int, lvl: int):
    a, b, c, d = _I32(), _I32(), _I32(), _I32()
    _check(lib().amgg_rs_level_size(h, lvl, C.byref(a), C.byref(b), C.byref(c), C.byref(d)), "amgg_rs_level_size")
    return a.value, b.value, c.value, d.value


def amgg_rs_copy_level(h: int, lvl: int, rowptr, col, val, p_rowptr=None, p_col=None, p_val=None, cf=None):
    _check(lib().amgg_rs_copy_level(h, lvl, _np_ptr(rowptr), _np_ptr(col), _np_ptr(val), _np_ptr(p_rowptr),
                                    _np_ptr(p_col), _np_ptr(p_val), _np_ptr(cf)), "amgg_rs_copy_level")


def amgg_rs_free(h: int):
    lib().amgg_rs_free(h)


def amgg_rs_begin(rowptr: np.ndarray, col: np.ndarray, val: np.ndarray, n: int, theta: float,
                  max_levels: int, max_coarse: int) -> int:
    rowptr = np.ascontiguousarray(rowptr, np.int32)
    col = np.ascontiguousarray(col, np.int32)
    val = np.ascontiguousarray(val, np.float64)
    h = _VP()
    _check(lib().amgg_rs_begin(_np_ptr(rowptr), _np_ptr(col), _np_ptr(val), n, theta, max_levels, max_coarse,
                               C.byref(h)), "amgg_rs_begin")
    return h.value


def amgg_rs_coarsen(h: int) -> bool:
    more = _I()
    _check(lib().amgg_rs_coarsen(h, C.byref(more)), "amgg_rs_coarsen")
    return bool(more.value)


def amgg_rs_galerkin(h: int):
    _check(lib().amgg_rs_galerkin(h), "amgg_rs_galerkin")


def amgg_rs_push_level(h: int, n: int, rowptr: np.ndarray, col: np.ndarray, val: np.ndarray):
    rowptr = np.ascontiguousarray(rowptr, np.int32)
    col = np.ascontiguousarray(col, np.int32)
    val = np.ascontiguousarray(val, np.float64)
    _check(lib().amgg_rs_push_level(h, n, _np_ptr(rowptr), _np_ptr(col), _np_ptr(val)), "amgg_rs_push_level")


def amgg_rs_setup_query(rowptr, col, val, n, theta=0.25, max_levels=10, max_coarse=500) -> amgg_hier_sizes:
    rowptr, col, val = (np.ascontiguousarray(a, t) for a, t in ((rowptr, np.int32), (col, np.int32), (val, np.float64)))
    z = amgg_hier_sizes()
    _check(lib().amgg_rs_setup_query(_np_ptr(rowptr), _np_ptr(col), _np_ptr(val), n, theta, max_levels, max_coarse,
                                     C.byref(z)), "amgg_rs_setup_query")
    return z


def amgg_rs_setup_fill(rowptr, col, val, n, theta, max_levels, max_coarse, levels):
    """levels: per level a dict of caller-allocated numpy arrays (rowptr, col, val, and p_rowptr,
    p_col, p_val above the coarsest level; cf optional), sized as amgg_rs_setup_query reported."""
    rowptr, col, val = (np.ascontiguousarray(a, t) for a, t in ((rowptr, np.int32), (col, np.int32), (val, np.float64)))
    out = amgg_hier_host()
    for l, arrs in enumerate(levels):
        for k, a in arrs.items():
            getattr(out, k)[l] = a.ctypes.data if a is not None else None
    _check(lib().amgg_rs_setup_fill(_np_ptr(rowptr), _np_ptr(col), _np_ptr(val), n, theta, max_levels, max_coarse,
                                    C.byref(out)), "amgg_rs_setup_fill")


def amgg_get_smoother_values(ctx, lvl, q_out, stream):
    return _check(lib().amgg_get_smoother_values(ctx, lvl, q_out, stream), "amgg_get_smoother_values")


def amgg_rs_split(h: int, strong: np.ndarray | None, cf_out: np.ndarray | None) -> int:
    """Split query (strong None) or C/F split from host strength flags (uint8, one per entry)."""
    more = _I()
    sp = None if strong is None else np.ascontiguousarray(strong, np.uint8)
    _check(lib().amgg_rs_split(h, _np_ptr(sp) if sp is not None else None,
                               _np_ptr(cf_out) if cf_out is not None else None, C.byref(more)), "amgg_rs_split")
    return more.value


def amgg_rs_push_interp(h: int, nc: int, rowptr: np.ndarray, col: np.ndarray, val: np.ndarray):
    rowptr = np.ascontiguousarray(rowptr, np.int32)
    col = np.ascontiguousarray(col, np.int32)
    val = np.ascontiguousarray(val, np.float64)
    _check(lib().amgg_rs_push_interp(h, nc, _np_ptr(rowptr), _np_ptr(col), _np_ptr(val)), "amgg_rs_push_interp")


# ---------------------------------------------------------------------------- device setup of a level
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
RELEASE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class TorchDeviceAllocator:
    """Allocator callbacks backed by torch tensors on one device (stream-ordered on torch's
    current stream, which is the stream the library is given)."""

    def __init__(self, torch, device):
        self.torch = torch
        self.device = device
        self.live = {}
        self.alloc = ALLOC_FN(self._alloc)
        self.release = RELEASE_FN(self._release)

    def _alloc(self, nbytes, user):
        try:
            t = self.torch.empty(max(int(nbytes), 1), dtype=self.torch.uint8, device=self.device)
        except RuntimeError:
            return None
        self.live[t.data_ptr()] = t
        return t.data_ptr()

    def _release(self, ptr, user):
        self.live.pop(ptr, None)

    def take(self, ptr, dtype, count):
        """The allocation at ptr as a tensor of `count` elements of `dtype`, owned by the caller."""
        t = self.live.pop(ptr)
        return t[: count * self.torch.empty(0, dtype=dtype).element_size()].view(dtype)


def amgg_strength_device(device: int, n: int, rowptr, col, val, theta: float, strong,
                         allocator: TorchDeviceAllocator | None = None):
    """Strength flags of a device CSR matrix into `strong` (uint8 tensor, one per entry)."""
    import torch

    dev = torch.device("cuda", device)
    al = allocator if allocator is not None else TorchDeviceAllocator(torch, dev)
    _check(lib().amgg_strength_device(device, n, rowptr.data_ptr(), col.data_ptr(), val.data_ptr(), int(col.numel()),
                                      float(theta), strong.data_ptr(), al.alloc, al.release, None,
                                      torch.cuda.current_stream(dev).cuda_stream), "amgg_strength_device")
    assert not al.live, "temporaries left allocated"
    return strong


def amgg_interp_device(device: int, n: int, rowptr, col, val, strong, cf, allocator: TorchDeviceAllocator | None = None):
    """Direct interpolation P of a device CSR matrix from device strength flags and C/F split
    (int8 tensor); returns (nc, (rowptr, col, val) tensors)."""
    import torch

    dev = torch.device("cuda", device)
    al = allocator if allocator is not None else TorchDeviceAllocator(torch, dev)
    nc, rp, cl, vl, nnz = _I32(), _VP(), _VP(), _VP(), _I32()
    _check(lib().amgg_interp_device(device, n, rowptr.data_ptr(), col.data_ptr(), val.data_ptr(), int(col.numel()),
                                    strong.data_ptr(), cf.data_ptr(), al.alloc, al.release, None, C.byref(nc),
                                    C.byref(rp), C.byref(cl), C.byref(vl), C.byref(nnz),
                                    torch.cuda.current_stream(dev).cuda_stream), "amgg_interp_device")
    out = (al.take(rp.value, torch.int32, n + 1), al.take(cl.value, torch.int32, nnz.value),
           al.take(vl.value, torch.float64, nnz.value))
    assert not al.live, "temporaries left allocated"
    return nc.value, out


def amgg_galerkin_device(device: int, n: int, nc: int, a_rowptr, a_col, a_val, p_rowptr, p_col, p_val,
                         chunk_products: int = 0, allocator: TorchDeviceAllocator | None = None):
    """A_c = P^T A P of device CSR tensors (int32 / float64); returns (rowptr, col, val) tensors."""
    import torch

    dev = torch.device("cuda", device)
    al = allocator if allocator is not None else TorchDeviceAllocator(torch, dev)
    rp, cl, vl, nnz = _VP(), _VP(), _VP(), _I32()
    _check(lib().amgg_galerkin_device(device, n, nc, a_rowptr.data_ptr(), a_col.data_ptr(), a_val.data_ptr(),
                                      int(a_col.numel()), p_rowptr.data_ptr(), p_col.data_ptr(), p_val.data_ptr(),
                                      int(p_col.numel()), al.alloc, al.release, None, int(chunk_products),
                                      C.byref(rp), C.byref(cl), C.byref(vl), C.byref(nnz),
                                      torch.cuda.current_stream(dev).cuda_stream), "amgg_galerkin_device")
    out = (al.take(rp.value, torch.int32, nc + 1), al.take(cl.value, torch.int32, nnz.value),
           al.take(vl.value, torch.float64, nnz.value))
    assert not al.live, "temporaries left allocated"
    return out


# ---------------------------------------------------------------------------- device context
def amgg_create(device: int, nlevels: int) -> int:
    c = _VP()
    _check(lib().amgg_create(C.byref(c), device, nlevels), "amgg_create")
    return c.value


def amgg_destroy(ctx: int):
    lib().amgg_destroy(ctx)


def amgg_load_level(ctx, lvl, n, nnz, rowptr, col, val):
    return _check(lib().amgg_load_level(ctx, lvl, n, nnz, rowptr, col, val), "amgg_load_level")


def amgg_load_prolong(ctx, lvl, n_f, n_c, nnz, rowptr, col, val):
    return _check(lib().amgg_load_prolong(ctx, lvl, n_f, n_c, nnz, rowptr, col, val), "amgg_load_prolong")


def amgg_workspace_bytes(ctx) -> int:
    b = C.c_size_t()
    _check(lib().amgg_workspace_bytes(ctx, C.byref(b)), "amgg_workspace_bytes")
    return b.value


def amgg_finalize(ctx, singular, workspace, ws_bytes, stream):
    return _check(lib().amgg_finalize(ctx, int(singular), workspace, ws_bytes, stream), "amgg_finalize")


def amgg_level_view_get(ctx, lvl) -> amgg_level_view:
    v = amgg_level_view()
    _check(lib().amgg_level_view_get(ctx, lvl, C.byref(v)), "amgg_level_view_get")
    return v


def amgg_set_smoother_coeffs(ctx, lvl, degree, coeffs, stream):
    c = np.ascontiguousarray(coeffs, np.float64)
    return _check(lib().amgg_set_smoother_coeffs(ctx, lvl, degree, _np_ptr(c), stream), "amgg_set_smoother_coeffs")


def amgg_set_smoother_coeffs_device(ctx, lvl, degree, coeffs_dev, stream):
    return _check(lib().amgg_set_smoother_coeffs_device(ctx, lvl, degree, coeffs_dev, stream),
                  "amgg_set_smoother_coeffs_device")


def amgg_set_smoother_coeffs_device_form(ctx, lvl, degree, coeffs_dev, diagonal, stream):
    return _check(lib().amgg_set_smoother_coeffs_device_form(ctx, lvl, degree, coeffs_dev, int(diagonal), stream),
                  "amgg_set_smoother_coeffs_device_form")


def amgg_set_smoother_jacobi(ctx, lvl, omega, stream):
    return _check(lib().amgg_set_smoother_jacobi(ctx, lvl, omega, stream), "amgg_set_smoother_jacobi")


def amgg_vcycle(ctx, nu1, nu2, precision, f, u, stream):
    return _check(lib().amgg_vcycle(ctx, nu1, nu2, precision, f, u, stream), "amgg_vcycle")


def amgg_level_apply(ctx, lvl, op, precision, x, y, f, stream):
    return _check(lib().amgg_level_apply(ctx, lvl, op, precision, x, y, f, stream), "amgg_level_apply")


def amgg_set_packed_columns(ctx, mode):
    return _check(lib().amgg_set_packed_columns(ctx, int(mode)), "amgg_set_packed_columns")


def amgg_set_fusion(ctx, enable):
    return _check(lib().amgg_set_fusion(ctx, int(enable)), "amgg_set_fusion")


def amgg_level_apply_timed(ctx, lvl, op, precision, x, y, f, start_event, stop_event, stream):
    return _check(lib().amgg_level_apply_timed(ctx, lvl, op, precision, x, y, f, start_event, stop_event, stream),
                  "amgg_level_apply_timed")


def amgg_solve(ctx, opts: amgg_solve_opts, b, x, history_cap: int, stream):
    info = amgg_solve_info()
    hist = np.zeros(max(history_cap, 1), np.float64)
    rc = _check(lib().amgg_solve(ctx, C.byref(opts), b, x, C.byref(info), _np_ptr(hist), history_cap, stream),
                "amgg_solve")
    return rc, info, hist


def amgg_judge_smoother(ctx, opts: amgg_solve_opts, iters, degree, coeffs_dev, diag_levels, b, x, stream):
    info = amgg_judge_info()
    _check(lib().amgg_judge_smoother(ctx, C.byref(opts), iters, degree, coeffs_dev, diag_levels, b, x, C.byref(info),
                                     stream), "amgg_judge_smoother")
    return info


def amgg_vcycle_loss_adjoint(ctx, nu1, nu2, precision, nvc, f, u0, loss_dev, dcoeffs_dev, stream):
    return _check(lib().amgg_vcycle_loss_adjoint(ctx, nu1, nu2, precision, nvc, f, u0, loss_dev, dcoeffs_dev,
                                                 stream), "amgg_vcycle_loss_adjoint")


def amgg_set_level_blocks(ctx, lvl, offsets, coeff_rows=None, singular=None):
    offsets = np.ascontiguousarray(offsets, np.int32)
    rows = None if coeff_rows is None else np.ascontiguousarray(coeff_rows, np.int32)
    sing = None if singular is None else np.ascontiguousarray(singular, np.int32)
    return _check(lib().amgg_set_level_blocks(ctx, lvl, offsets.size - 1, _np_ptr(offsets), _np_ptr(rows),
                                              _np_ptr(sing)), "amgg_set_level_blocks")


def amgg_set_smoother_coeffs_blocks(ctx, lvl, degree, coeffs_dev, stride, stream):
    return _check(lib().amgg_set_smoother_coeffs_blocks(ctx, lvl, degree, coeffs_dev, stride, stream),
                  "amgg_set_smoother_coeffs_blocks")


def amgg_set_smoother_coeffs_blocks_form(ctx, lvl, degree, coeffs_dev, stride, diagonal, stream):
    return _check(lib().amgg_set_smoother_coeffs_blocks_form(ctx, lvl, degree, coeffs_dev, stride, int(diagonal),
                                                             stream),
                  "amgg_set_smoother_coeffs_blocks_form")


def amgg_vcycle_loss_adjoint_blocks(ctx, nu1, nu2, precision, nvc, f, u0, loss_dev, dcoeffs_dev, dcoeff_rows,
                                    stream):
    return _check(lib().amgg_vcycle_loss_adjoint_blocks(ctx, nu1, nu2, precision, nvc, f, u0, loss_dev, dcoeffs_dev,
                                                        dcoeff_rows, stream), "amgg_vcycle_loss_adjoint_blocks")


def amgg_chain_loss_grad(nrows, ncols, dcoeffs, row_problem, dloss, out, stream):
    return _check(lib().amgg_chain_loss_grad(nrows, ncols, dcoeffs, row_problem, dloss, out, stream),
                  "amgg_chain_loss_grad")


def amgg_validation_metric(n, loss, loss_jacobi, out, stream):
    return _check(lib().amgg_validation_metric(n, loss, loss_jacobi, out, stream), "amgg_validation_metric")


def amgg_cast_scale_f64_f32(src, dst, n, scale, stream):
    return _check(lib().amgg_cast_scale_f64_f32(src, dst, n, scale, stream), "amgg_cast_scale_f64_f32")


# ---------------------------------------------------------------------------- GCIN predictor
def gcin_param_count(degree: int, hidden: int = 64) -> int:
    v = lib().gcin_param_count_hidden(degree, hidden)
    if v < 0:
        raise AmggError(AMGG_EINVAL, "gcin_param_count: degree or hidden width out of range")
    return v


def gcin_batch_workspace_bytes(n, nnz, hidden: int = 64, flags: int = 0) -> int:
    n = np.ascontiguousarray(n, np.int32)
    nnz = np.ascontiguousarray(nnz, np.int32)
    b = C.c_size_t()
    _check(lib().gcin_batch_workspace_bytes_ex(hidden, flags, n.size, _np_ptr(n), _np_ptr(nnz), C.byref(b)),
           "gcin_batch_workspace_bytes")
    return b.value


def gcin_batch_create(graphs, workspace, ws_bytes, stream, hidden: int = 64, flags: int = 0) -> int:
    """graphs: list of (n, nnz, rowptr_ptr, col_ptr, val_ptr) device CSR views."""
    arr = (gcin_graph * len(graphs))(*[gcin_graph(*g) for g in graphs])
    h = _VP()
    _check(lib().gcin_batch_create_ex(hidden, flags, len(graphs), arr, workspace, ws_bytes, stream, C.byref(h)),
           "gcin_batch_create")
    return h.value


def gcin_batch_destroy(b):
    lib().gcin_batch_destroy(b)


def gcin_forward(b, degree, precision, params, coeffs_out, stream):
    return _check(lib().gcin_forward(b, degree, precision, params, coeffs_out, stream), "gcin_forward")


def gcin_backward(b, degree, precision, params, dcoeffs, grads, stream):
    return _check(lib().gcin_backward(b, degree, precision, params, dcoeffs, grads, stream), "gcin_backward")


def adam_scratch_bytes() -> int:
    return lib().adam_scratch_bytes()


def adam_step(params, grads, m, v, n, lr, b1, b2, eps, step, clip, gnorm_out, scratch, stream):
    return _check(lib().adam_step(params, grads, m, v, n, lr, b1, b2, eps, step, clip, gnorm_out, scratch, stream),
                  "adam_step")


def adam_step_noalloc(params, grads, m, v, n, lr, b1, b2, eps, step, clip, gnorm_out, stream):
    return _check(lib().adam_step_noalloc(params, grads, m, v, n, lr, b1, b2, eps, step, clip, gnorm_out, stream),
                  "adam_step_noalloc")


def gcin_tile_gemm_check(A, B, D_fp32, D_bf16, stream):
    return _check(lib().gcin_tile_gemm_check(A, B, D_fp32, D_bf16, stream), "gcin_tile_gemm_check")
