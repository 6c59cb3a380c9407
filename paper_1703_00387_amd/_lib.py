"""ctypes binding of libmps.so (argument marshalling only).

Every entry point of include/mps.h is exposed under the same name.  Tensors
are passed as raw device pointers (``tensor.data_ptr()``) and the current
PyTorch HIP stream (``torch.cuda.current_stream().cuda_stream``).  The
library must have been built (``python -m paper_1703_00387_amd.build``); if it
is missing the import fails loudly -- there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmps.so")

MPS_OK, MPS_ERR_INVALID, MPS_ERR_SHAPE, MPS_ERR_CAPACITY, MPS_ERR_NOCONV, MPS_ERR_NONFINITE, \
    MPS_ERR_HIP, MPS_ERR_UNSUPPORTED = range(8)
STATUS_NAMES = {0: "MPS_OK", 1: "MPS_ERR_INVALID", 2: "MPS_ERR_SHAPE", 3: "MPS_ERR_CAPACITY",
                4: "MPS_ERR_NOCONV", 5: "MPS_ERR_NONFINITE", 6: "MPS_ERR_HIP", 7: "MPS_ERR_UNSUPPORTED"}
MPS_DEV_NOCONV_SVD, MPS_DEV_NOCONV_LANCZOS, MPS_DEV_NONFINITE, MPS_DEV_SCHED_TIMEOUT = 0x1, 0x2, 0x4, 0x8
MPS_DEV_CHARGE = 0x10
MPS_FLAG_GRAPH, MPS_FLAG_FIXED_SWEEPS, MPS_FLAG_PLAIN, MPS_FLAG_CHECKPOINT, MPS_FLAG_OBSERVE = 0x1, 0x2, 0x4, 0x8, 0x10
MPS_C64, MPS_C128 = 0, 1
MPS_OP_TRUNCATE, MPS_OP_TEBD, MPS_OP_HEFF, MPS_OP_KRYLOV, MPS_OP_TDVP = range(5)

# every exported symbol that include/mps.h declares
EXPORTS = ["mps_create", "mps_create_ws", "mps_workspace_size", "mps_workspace_needed", "mps_destroy", "mps_last_error", "mps_reserve", "mps_device_status",
           "mps_set_option", "mps_kernel_stats", "mps_gates", "mps_truncate", "mps_truncate_ex", "mps_truncate_noalloc", "mps_truncate_u1", "mps_tebd_step", "mps_tebd_step_ex", "mps_tebd_ckpt_bytes", "mps_tebd_step_vjp", "mps_theta_gate_vjp", "mps_truncate_vjp", "mps_tebd_step_u1", "mps_ktebd_step", "mps_ktebd_step_u1", "mps_tebd_td_step", "mps_tebd_td_step_u1", "mps_cfme_nodes",
           "mps_observe", "mps_heff_apply", "mps_krylov_expm", "mps_env_update", "mps_tdvp2_step", "mps_tdvp2_step_u1",
           "mps_tebd_grad_arena_bytes", "mps_tebd_grad", "mps_tebd_vjp", "mps_autotune_jacobi",
           "mps_autotune_candidate", "mps_autotune_gemm", "mps_gemm_candidate", "mps_gemm_tile_choice",
           "mps_set_gemm_tile"]


class ChainDesc(C.Structure):
    _fields_ = [("L", C.c_int32), ("d", C.c_int32), ("chi_max", C.c_int32), ("dtype", C.c_int32),
                ("B", C.c_void_p), ("lam", C.c_void_p), ("chi", C.c_void_p), ("hbond", C.c_void_p),
                ("disc", C.c_void_p)]


class U1ChainDesc(C.Structure):
    _fields_ = [("qbond", C.c_void_p), ("qsite", C.c_int32 * 5), ("modulus", C.c_int32), ("reserved", C.c_int32 * 2)]


class OCChainDesc(C.Structure):
    _fields_ = [("L", C.c_int32), ("d", C.c_int32), ("chi_max", C.c_int32), ("dtype", C.c_int32),
                ("w", C.c_int32), ("reserved", C.c_int32), ("M", C.c_void_p), ("chi", C.c_void_p), ("W", C.c_void_p)]


class MPSError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load libmps.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1703_00387_amd.build`")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, dbl, u32 = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_uint32
    sig = {
        "mps_create": [C.POINTER(vp), C.c_int],
        "mps_create_ws": [C.POINTER(vp), C.c_int, vp, C.c_size_t],
        "mps_workspace_size": [i32, i32, i32, i32, i32, i32, i32, i32],
        "mps_workspace_needed": [vp, C.POINTER(C.c_size_t)],
        "mps_destroy": [vp],
        "mps_reserve": [vp, C.c_size_t],
        "mps_device_status": [vp, vp, C.POINTER(u32)],
        "mps_set_option": [vp, C.c_int, dbl],
        "mps_kernel_stats": [vp, vp, i32, C.POINTER(dbl), C.POINTER(i64), C.POINTER(C.c_uint64), i32],
        "mps_gates": [vp, vp, i32, i32, vp, vp, vp, vp],
        "mps_truncate": [vp, vp, vp, i64, i64, i64, dbl, vp, vp, vp, vp, vp, vp],
        "mps_truncate_noalloc": [vp, vp, vp, i64, i64, i64, dbl, vp, vp, vp, vp, vp, vp],
        "mps_truncate_u1": [vp, vp, vp, i64, i64, vp, vp, i64, dbl, vp, vp, vp, vp, vp, vp, vp],
        "mps_tebd_step": [vp, vp, C.POINTER(ChainDesc), i32, i32, dbl, i32, dbl, u32],
        "mps_tebd_step_ex": [vp, vp, C.POINTER(ChainDesc), i32, i32, dbl, i32, dbl, u32, vp, C.c_size_t, vp, vp, vp],
        "mps_truncate_ex": [vp, vp, i32, vp, i64, i64, i64, dbl, i32, vp, vp, vp, vp, vp, vp],
        "mps_tebd_step_vjp": [vp, vp, C.POINTER(ChainDesc), i32, C.POINTER(vp), vp, C.c_size_t, C.POINTER(vp),
                              C.POINTER(vp), vp, dbl],
        "mps_theta_gate_vjp": [vp, vp, vp, vp, vp, vp, vp, i32, i32, i32, i32, vp, vp, vp, vp],
        "mps_truncate_vjp": [vp, vp, vp, i64, i64, i32, vp, vp, vp, i64, vp, vp, dbl, vp],
        "mps_tebd_step_u1": [vp, vp, C.POINTER(ChainDesc), C.POINTER(U1ChainDesc), i32, i32, dbl, i32, dbl, u32],
        "mps_ktebd_step_u1": [vp, vp, C.POINTER(ChainDesc), C.POINTER(U1ChainDesc), i32, dbl, i32, dbl, i32, dbl, u32,
                              vp],
        "mps_ktebd_step": [vp, vp, C.POINTER(ChainDesc), i32, dbl, i32, dbl, i32, dbl, u32, vp],
        "mps_tebd_td_step_u1": [vp, vp, C.POINTER(ChainDesc), C.POINTER(U1ChainDesc), i32, i32, dbl, i32, dbl, u32,
                                i32, i32, vp, vp],
        "mps_tebd_td_step": [vp, vp, C.POINTER(ChainDesc), i32, i32, dbl, i32, dbl, u32, i32, i32, vp, vp],
        "mps_cfme_nodes": [i32, vp, vp],
        "mps_autotune_jacobi": [vp, vp, i32, i32, i32, i32, vp, vp, vp],
        "mps_autotune_candidate": [i32, i32, vp, vp, vp],
        "mps_autotune_gemm": [vp, vp, i32, i32, i32, i32, i32, i32, i32, vp, vp, vp],
        "mps_gemm_candidate": [i32, vp, vp],
        "mps_gemm_tile_choice": [i32, i32, i32, i32, vp],
        "mps_set_gemm_tile": [i32, i32, i32, i32, i32],
        "mps_observe": [vp, vp, C.POINTER(ChainDesc), vp, vp, vp, i32, vp, vp],
        "mps_heff_apply": [vp, vp, i32, vp, vp, vp, vp, vp, vp, i64, i32, i32, i64, i32, i32, i32],
        "mps_krylov_expm": [vp, vp, i32, vp, vp, vp, vp, vp, i64, i32, i32, i64, i32, i32, i32, dbl, dbl, i32, dbl,
                            vp, vp],
        "mps_env_update": [vp, vp, i32, i32, vp, vp, vp, vp, i64, i32, i64, i32, i32],
        "mps_tdvp2_step_u1": [vp, vp, C.POINTER(OCChainDesc), C.POINTER(U1ChainDesc), dbl, i32, dbl, i32, dbl, vp, vp],
        "mps_tdvp2_step": [vp, vp, C.POINTER(OCChainDesc), dbl, i32, dbl, i32, dbl, vp, vp],
        "mps_tebd_grad": [vp, vp, C.POINTER(ChainDesc), vp, dbl, i32, dbl, dbl, vp, i32, vp, vp, C.c_size_t, vp, vp],
        "mps_tebd_vjp": [vp, vp, C.POINTER(ChainDesc), vp, dbl, i32, dbl, dbl, vp, vp, vp, vp, vp, C.c_size_t, vp, vp],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = C.c_int
    L.mps_tebd_grad_arena_bytes.argtypes = [i32, i32, i32, i32]
    L.mps_tebd_grad_arena_bytes.restype = C.c_size_t
    L.mps_workspace_size.restype = C.c_size_t
    L.mps_tebd_ckpt_bytes.argtypes = [C.POINTER(ChainDesc), i32, i32]
    L.mps_tebd_ckpt_bytes.restype = C.c_size_t
    L.mps_last_error.argtypes = [vp]
    L.mps_last_error.restype = C.c_char_p
    _lib = L
    return L


def check(h, code):
    if code != MPS_OK:
        msg = lib().mps_last_error(h)
        raise MPSError(code, msg.decode() if msg else "")
    return code
