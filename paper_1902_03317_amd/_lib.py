"""ctypes binding of libpasta.so (declarations in include/pasta.h).

Argument marshalling only: every computation runs in the HIP library. If the
library is missing this module raises at import; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# PASTA_LIBRARY may name another build of the same library (e.g. one compiled
# with different tuning parameters); by default the in-tree build is used.
LIB_PATH = os.environ.get("PASTA_LIBRARY") or os.path.join(HERE, "libpasta.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_1902_03317_amd.build` "
                      "(or __graft_entry__.build()) first")

lib = ctypes.CDLL(LIB_PATH)

P = ctypes.c_void_p
U32 = ctypes.c_uint32
U64 = ctypes.c_uint64
SZ = ctypes.c_size_t
F32 = ctypes.c_float

PASTA_F32 = 0
PASTA_BF16 = 1
EWOP = {"add": 0, "sub": 1, "mul": 2, "div": 3}
STATUS = {0: "PASTA_OK", 1: "PASTA_EINVAL", 2: "PASTA_ERANGE", 3: "PASTA_EUNSUPPORTED", 4: "PASTA_EWORKSPACE",
          5: "PASTA_EHIP", 6: "PASTA_EINTERNAL"}

# name -> argtypes; every entry point returns pasta_status (int)
SIGNATURES = {
    "pasta_coo_workspace_bytes": [U32, P, U64, ctypes.POINTER(SZ)],
    "pasta_coo_create": [U32, P, U64, P, P, P, SZ, P, ctypes.POINTER(P)],
    "pasta_coo_destroy": [P],
    "pasta_coo_check": [P, P],
    "pasta_coo_info": [P, ctypes.POINTER(U32), ctypes.POINTER(U64)],
    "pasta_coo_mode_view": [P, U32, ctypes.POINTER(P), ctypes.POINTER(P), P, ctypes.POINTER(P)],
    "pasta_mttkrp_workspace_bytes": [P, U32, U32, ctypes.c_int, ctypes.POINTER(SZ)],
    "pasta_mttkrp": [P, U32, P, ctypes.c_int, U32, U32, P, F32, P, U32, P, SZ, P],
    "pasta_mttkrp_atomic": [P, U32, P, ctypes.c_int, U32, U32, P, U32, P],
    "pasta_mttkrp_static": [P, U32, P, ctypes.c_int, U32, U32, P, F32, P, U32, P],
    "pasta_cp_sample": [P, P, ctypes.c_int, U32, U32, P, P],
    "pasta_cp_workspace_bytes": [P, U32, ctypes.c_int, ctypes.POINTER(SZ)],
    "pasta_cp_residual_loss": [P, P, ctypes.c_int, U32, U32, P, P, P, SZ, P],
    "pasta_cp_grad_workspace_bytes": [P, U32, ctypes.c_int, ctypes.POINTER(SZ)],
    "pasta_cp_grad": [P, P, ctypes.c_int, U32, U32, F32, P, U32, P, P, SZ, P],
    "pasta_cast_f32_to_bf16": [P, P, U64, P],
    "pasta_scale_f32": [P, U64, P, P],
    "pasta_probe_gather": [P, U32, U32, U32, U32, U32, U32, P, P],
    "pasta_arm_kernel_events": [P, P],
    "pasta_set_mttkrp_form": [ctypes.c_int],
    "pasta_last_mttkrp_form": [P],
    "pasta_cp_als_workspace_bytes": [P, U32, ctypes.POINTER(SZ)],
    "pasta_cp_als_sweep": [P, P, U32, U32, P, P, P, P, SZ, P],
    "pasta_adam_step": [P, P, P, P, P, U64, F32, F32, F32, F32, U32, P],
    "pasta_fibers_workspace_bytes": [P, U32, ctypes.POINTER(SZ)],
    "pasta_fibers_create": [P, U32, P, SZ, P, ctypes.POINTER(P)],
    "pasta_fibers_destroy": [P],
    "pasta_fibers_info": [P, ctypes.POINTER(U32), ctypes.POINTER(U64)],
    "pasta_fibers_view": [P, ctypes.POINTER(P), P, ctypes.POINTER(P), ctypes.POINTER(P)],
    "pasta_ttm_workspace_bytes": [P, U32, ctypes.c_int, ctypes.POINTER(SZ)],
    "pasta_ttm": [P, P, ctypes.c_int, U32, U32, P, U32, P, SZ, P],
    "pasta_ttv_workspace_bytes": [P, ctypes.POINTER(SZ)],
    "pasta_ttv": [P, P, P, P, SZ, P],
    "pasta_tew_eq": [ctypes.c_int, U64, P, P, P, P],
    "pasta_ts": [ctypes.c_int, U64, P, F32, P, P],
    "pasta_tew_workspace_bytes": [U32, U64, U64, ctypes.POINTER(SZ)],
    "pasta_tew": [U32, ctypes.c_int, P, U64, P, P, P, U64, P, P, P, P, P, ctypes.POINTER(U64), P, SZ, P],
}

for _name, _args in SIGNATURES.items():
    _f = getattr(lib, _name)
    _f.argtypes = _args
    _f.restype = ctypes.c_int

lib.pasta_status_str.argtypes = [ctypes.c_int]
lib.pasta_status_str.restype = ctypes.c_char_p
lib.pasta_last_hip_error.argtypes = []
lib.pasta_last_hip_error.restype = ctypes.c_int

EXPORTS = sorted(list(SIGNATURES) + ["pasta_status_str", "pasta_last_hip_error"])


class PastaError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = lib.pasta_status_str(status).decode()
        extra = f" (hipError {lib.pasta_last_hip_error()})" if status == 5 else ""
        super().__init__(f"{where}: {STATUS.get(status, status)}: {msg}{extra}")


def check(status: int, where: str) -> None:
    if status != 0:
        raise PastaError(status, where)


def ptr_array(ptrs):
    arr = (ctypes.c_void_p * len(ptrs))()
    for i, p in enumerate(ptrs):
        arr[i] = p
    return arr
