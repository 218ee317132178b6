"""ctypes declarations of the C ABI in include/rsvd.h (librsvd.so, built in-tree).

Loading fails loudly: there is no fallback implementation of any kind.
"""

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librsvd.so")

# status codes (rsvd_status)
RSVD_OK = 0
RSVD_E_INVAL = 1
RSVD_E_WORKSPACE = 2
RSVD_E_DEVICE = 3
RSVD_E_UNSUPPORTED = 4
RSVD_E_BREAKDOWN = 5
RSVD_E_NONFINITE = 6
RSVD_E_NOCONV = 7

# enums
RSVD_F32, RSVD_F64 = 0, 1
RSVD_GAUSSIAN, RSVD_SRFT, RSVD_GSRFT = 0, 1, 2
RSVD_NATIVE, RSVD_BF16, RSVD_BF16X3 = 0, 1, 2
RSVD_FLAG_SHIFTED, RSVD_FLAG_NONFINITE, RSVD_FLAG_NOCONV = 1, 2, 4
RSVD_MAX_L = 128
RSVD_STATIC_SCRATCH_BYTES = 32 << 20

EXPORTS = [
    "rsvd_create", "rsvd_destroy", "rsvd_validate", "rsvd_workspace_bytes", "rsvd_status_string",
    "rsvd_range_finder", "rsvd_power_iter", "rsvd_project", "rsvd_svd",
    "rsvd_batched_workspace_bytes", "rsvd_batched", "rsvd_backward_workspace_bytes", "rsvd_backward",
    "rsvd_backward_batched_workspace_bytes", "rsvd_backward_batched", "rsvd_forward_kept", "rsvd_backward_kept",
    "rsvd_batched_kept", "rsvd_backward_batched_kept", "rsvd_full_workspace_bytes", "rsvd_full",
    "rsvd_full_static", "rsvd_range_finder_tol_workspace_bytes", "rsvd_range_finder_tol",
    "rsvd_sketch", "rsvd_draw_omega", "rsvd_draw_srft", "rsvd_orth", "rsvd_device_status",
    "rsvd_profile_enable", "rsvd_profile_select", "rsvd_profile_read", "rsvd_probe_hbm_read", "rsvd_probe_mfma",
    "rsvd_eigh", "rsvd_nystrom", "rsvd_eigh_onepass", "rsvd_svd_onepass",
]
KERNEL_KINDS = ["stream_nn", "stream_tn", "small_gemm", "gram", "chol", "jacobi", "pack", "srft", "eig", "gsrft"]


class RsvdProblem(ctypes.Structure):
    """Mirror of `rsvd_problem` (include/rsvd.h)."""
    _fields_ = [
        ("m", ctypes.c_int64), ("n", ctypes.c_int64), ("lda", ctypes.c_int64),
        ("k", ctypes.c_int32), ("p", ctypes.c_int32), ("q", ctypes.c_int32),
        ("dtype", ctypes.c_int32), ("sketch", ctypes.c_int32), ("prec", ctypes.c_int32),
        ("seed", ctypes.c_uint64), ("stream_id", ctypes.c_uint64),
    ]


class RsvdError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        super().__init__(f"{where}: {status_string(status)} (status {status})")


_lib = None


def load():
    """Load librsvd.so once and declare every exported signature."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -m paper_0909_4061_amd.build` "
            "(the randomized SVD has no non-HIP implementation)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, sz, i32, i64 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_int64
    prob = ctypes.POINTER(RsvdProblem)
    sig = {
        "rsvd_create": ([ctypes.POINTER(vp), ctypes.c_int], i32),
        "rsvd_destroy": ([vp], i32),
        "rsvd_validate": ([prob], i32),
        "rsvd_workspace_bytes": ([prob], sz),
        "rsvd_status_string": ([i32], ctypes.c_char_p),
        "rsvd_range_finder": ([vp, prob, vp, vp, vp, sz, vp], i32),
        "rsvd_power_iter": ([vp, prob, vp, vp, vp, sz, vp], i32),
        "rsvd_project": ([vp, prob, vp, vp, vp, vp, sz, vp], i32),
        "rsvd_svd": ([vp, prob, vp, vp, vp, vp, vp, vp, sz, vp], i32),
        "rsvd_eigh": ([vp, prob, vp, vp, vp, vp, vp, sz, vp], i32),
        "rsvd_nystrom": ([vp, prob, vp, vp, vp, vp, vp, sz, vp], i32),
        "rsvd_eigh_onepass": ([vp, prob, vp, vp, vp, vp, sz, vp], i32),
        "rsvd_svd_onepass": ([vp, prob, vp, vp, vp, vp, vp, sz, vp], i32),
        "rsvd_sketch": ([vp, prob, vp, vp, vp, sz, vp], i32),
        "rsvd_batched_workspace_bytes": ([i32, prob], sz),
        "rsvd_backward_workspace_bytes": ([prob], sz),
        "rsvd_backward": ([vp, prob, vp, vp, vp, vp, vp, vp, sz, vp], i32),
        "rsvd_batched": ([vp, i32, prob, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp),
                          ctypes.POINTER(vp), vp, sz, vp], i32),
        "rsvd_backward_batched_workspace_bytes": ([i32, prob], sz),
        "rsvd_backward_batched": ([vp, i32, prob] + [ctypes.POINTER(vp)] * 5 + [vp, sz, vp], i32),
        "rsvd_backward_batched_kept": ([vp, i32, prob] + [ctypes.POINTER(vp)] * 5 + [vp, sz, vp], i32),
        "rsvd_batched_kept": ([vp, i32, prob] + [ctypes.POINTER(vp)] * 4 + [vp, sz, vp], i32),
        "rsvd_forward_kept": ([vp, prob, vp, vp, vp, vp, vp, sz, vp], i32),
        "rsvd_full_workspace_bytes": ([prob], sz),
        "rsvd_full": ([vp, prob, vp, vp, vp, vp, vp, sz, vp], i32),
        "rsvd_full_static": ([vp, prob, vp, vp, vp, vp, vp], i32),
        "rsvd_range_finder_tol_workspace_bytes": ([prob, i32], sz),
        "rsvd_range_finder_tol": ([vp, prob, ctypes.c_double, i32, vp, vp, ctypes.POINTER(i32),
                                   ctypes.POINTER(ctypes.c_double), vp, sz, vp], i32),
        "rsvd_backward_kept": ([vp, prob, vp, vp, vp, vp, vp, vp, sz, vp], i32),
        "rsvd_draw_omega": ([vp, prob, vp, vp], i32),
        "rsvd_draw_srft": ([vp, prob, vp, vp, vp], i32),
        "rsvd_orth": ([vp, prob, i64, vp, vp, vp, sz, vp], i32),
        "rsvd_device_status": ([vp, vp, ctypes.POINTER(i32)], i32),
        "rsvd_profile_enable": ([vp, i32], i32),
        "rsvd_profile_select": ([vp, ctypes.c_uint32], i32),
        "rsvd_profile_read": ([vp, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double)], i32),
        "rsvd_probe_hbm_read": ([vp, sz, vp, vp], i32),
        "rsvd_probe_mfma": ([i32, i64, i64, vp, vp], i32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def status_string(status):
    try:
        return load().rsvd_status_string(int(status)).decode()
    except ImportError:
        return "library not loaded"


def check(status, where):
    if status != RSVD_OK:
        raise RsvdError(status, where)
