"""ctypes binding of libmm.so (the C ABI of include/mm.h).

Argument marshalling only: every computation runs in the library's HIP
kernels.  Device buffers are torch tensors on the current HIP device; their
data pointers and the current stream are handed to the library.  There is
no fallback: if libmm.so is missing or cannot be loaded, importing the
binding fails.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmm.so")

MM_OK = 0
STATUS = {0: "MM_OK", 1: "MM_E_INVALID", 2: "MM_E_NOMEM", 3: "MM_E_NOT_SPD",
          4: "MM_E_NO_CONVERGE", 5: "MM_E_STATE", 6: "MM_E_DEVICE"}
MM_MODAL = 0
MM_CHOLESKY = 1
MM_STEP_EXACT = 1
MM_STEP_SCAN = 2

# Every exported entry point of include/mm.h.
SYMBOLS = ["mm_setup", "mm_decompose", "mm_decompose_projected", "mm_step_modal", "mm_step_modal_noalloc", "mm_step_modal_exact", "mm_step_modal_scan", "mm_modal_phasors", "mm_select_modes", "mm_step_modal_selective", "mm_step_cholesky",
           "mm_probe", "mm_reset_state", "mm_get_state", "mm_set_state", "mm_eigenvalues", "mm_info",
           "mm_destroy", "mm_last_error", "mm_batch_create", "mm_batch_run",
           "mm_batch_info", "mm_batch_destroy", "mm_adjoint_modal", "mmk_dgemm", "mmk_dgemm_tri", "mmk_dsymm_lower", "mmk_dpotrf",
           "mmk_dtrtri", "mmk_dsy2sb", "mmk_dsb2st", "mmk_dstedc", "mmk_dsyevd"]


class MMError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Problem(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("xyz", ctypes.c_void_p), ("h", ctypes.c_double),
                ("r_nnz", ctypes.c_int64), ("r_rowptr", ctypes.c_void_p),
                ("r_col", ctypes.c_void_p), ("r_val", ctypes.c_void_p),
                ("n_e", ctypes.c_int32), ("e_nnz", ctypes.c_int64),
                ("e_rowptr", ctypes.c_void_p), ("e_col", ctypes.c_void_p),
                ("e_val", ctypes.c_void_p), ("n_src", ctypes.c_int32),
                ("M0", ctypes.c_void_p), ("n_probe", ctypes.c_int32),
                ("P", ctypes.c_void_p), ("L", ctypes.c_void_p), ("ldl", ctypes.c_int64)]


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libmm.so and declare the signatures (no GPU work)."""
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with "
                          "`python -m paper_2407_11993_amd.build`")
    lib = ctypes.CDLL(path)
    vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    sigs = {
        "mm_setup": [ctypes.POINTER(Problem), vp, ctypes.POINTER(vp)],
        "mm_decompose": [vp],
        "mm_decompose_projected": [vp],
        "mm_step_modal": [vp, dbl, dbl, i64, vp, vp, vp],
        "mm_step_modal_noalloc": [vp, dbl, dbl, i64, vp, vp, vp],
        "mm_step_modal_exact": [vp, dbl, i64, vp, vp, vp],
        "mm_modal_phasors": [vp, i64, vp, vp, vp, vp],
        "mm_step_modal_scan": [vp, dbl, i32, dbl, i64, vp, vp, vp],
        "mm_select_modes": [vp, dbl, ctypes.POINTER(ctypes.c_int64), vp],
        "mm_step_modal_selective": [vp, dbl, ctypes.c_uint32, dbl, i64, vp, vp, vp],
        "mm_step_cholesky": [vp, dbl, dbl, i64, vp, vp, vp],
        "mm_probe": [vp, i32, i32, vp, vp],
        "mm_reset_state": [vp],
        "mm_get_state": [vp, i32, vp],
        "mm_set_state": [vp, i32, vp],
        "mm_eigenvalues": [vp, vp],
        "mm_info": [vp, ctypes.POINTER(ctypes.c_int64)],
        "mm_destroy": [vp],
        "mm_last_error": [vp],
        "mm_batch_create": [vp, dbl, dbl, i32, ctypes.POINTER(ctypes.c_int64),
                            ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                            vp, vp, i32, ctypes.POINTER(vp)],
        "mm_batch_run": [vp],
        "mm_batch_info": [vp, ctypes.POINTER(ctypes.c_int64)],
        "mm_batch_destroy": [vp],
        "mm_adjoint_modal": [vp, dbl, dbl, i64, i32, ctypes.POINTER(ctypes.c_int32),
                             ctypes.POINTER(ctypes.c_int32), vp, vp, i64, vp, vp, vp],
        "mmk_dgemm": [i32, i32, i64, i64, i64, dbl, vp, i64, vp, i64, dbl, vp, i64, vp],
        "mmk_dgemm_tri": [i32, i32, i64, i64, i64, dbl, vp, i64, vp, i64, dbl, vp, i64, i32, i64, vp],
        "mmk_dsymm_lower": [i64, i64, dbl, vp, i64, vp, i64, dbl, vp, i64, vp],
        "mmk_dpotrf": [i64, vp, i64, ctypes.POINTER(ctypes.c_int64), vp],
        "mmk_dtrtri": [i64, vp, i64, vp],
        "mmk_dsy2sb": [i64, vp, i64, i32, vp, i64, vp],
        "mmk_dsb2st": [i64, i32, vp, i64, vp, vp, vp],
        "mmk_dstedc": [i64, vp, vp, vp, vp, vp],
        "mmk_dsyevd": [i64, vp, i64, i32, vp, vp, vp],
    }
    for name, args in sigs.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = None if name in ("mm_destroy", "mm_batch_destroy") else (
            ctypes.c_char_p if name == "mm_last_error" else ctypes.c_int)
    return lib


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        _lib = load()
    return _lib


def check(code: int, ctx=None) -> None:
    if code != MM_OK:
        msg = lib().mm_last_error(ctx)
        raise MMError(code, msg.decode() if msg else "")


def ptr(t) -> int | None:
    """Device pointer of a torch tensor (None for None)."""
    if t is None:
        return None
    return t.data_ptr()


def stream_handle():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
