"""ctypes declarations of libfvpcg.so (include/fvpcg.h).

torch is imported first so that the library binds to the HIP runtime torch
already loaded (both carry the soname libamdhip64.so.7): device pointers and
streams from torch are then valid inside the library.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfvpcg.so")

OK, NOT_CONVERGED, INVALID_ARG, INVALID_MESH, BREAKDOWN, DEVICE_ERROR, OUT_OF_MEMORY, UNSUPPORTED = 0, 1, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "OK", 1: "NOT_CONVERGED", -1: "INVALID_ARG", -2: "INVALID_MESH", -3: "BREAKDOWN",
                -4: "DEVICE_ERROR", -5: "OUT_OF_MEMORY", -6: "UNSUPPORTED"}
CG, PIPECG, PIPECG_LITERAL = 0, 1, 2
PRECOND_NONE, PRECOND_JACOBI = 0, 1
FP32_COPY = 1
PSOLVER_JACOBI, PSOLVER_AMG = 0, 1
MAX_ROW_DEGREE = 32

# Every function the header declares, with (restype, argtypes).
P = ctypes.c_void_p
i32 = ctypes.c_int32
u32 = ctypes.c_uint32
u64 = ctypes.c_uint64
f64 = ctypes.c_double
PP = ctypes.POINTER(ctypes.c_void_p)


class Stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("outer_iters", ctypes.c_int32), ("status", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("rel_res", ctypes.c_double), ("true_rel_res", ctypes.c_double),
                ("r0_norm", ctypes.c_double), ("b_norm", ctypes.c_double), ("device_ms", ctypes.c_double),
                ("iter_ms", ctypes.c_double)]

    def asdict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}
        d["status_name"] = STATUS_NAMES.get(self.status, str(self.status))
        return d


SPS = ctypes.POINTER(Stats)

SIGNATURES = {
    "fvpcg_version": (ctypes.c_int, []),
    "fvpcg_last_error": (ctypes.c_char_p, []),
    "fvpcg_mesh_create": (ctypes.c_int, [i32, i32, P, P, P, PP]),
    "fvpcg_mesh_destroy": (ctypes.c_int, [P]),
    "fvpcg_mesh_info": (ctypes.c_int, [P, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32)]),
    "fvpcg_matrix_create": (ctypes.c_int, [P, P, P, P, u32, P, PP]),
    "fvpcg_matrix_update": (ctypes.c_int, [P, P, P, P, P]),
    "fvpcg_matrix_destroy": (ctypes.c_int, [P]),
    "fvpcg_spmv": (ctypes.c_int, [P, P, P, P]),
    "fvpcg_solve": (ctypes.c_int, [P, P, P, f64, i32, i32, i32, P, SPS]),
    "fvpcg_solve_noalloc": (ctypes.c_int, [P, P, P, f64, i32, i32, i32, P, SPS]),
    "fvpcg_solve_bicgstab": (ctypes.c_int, [P, P, P, f64, i32, i32, P, SPS]),
    "fvpcg_solve_bicgstab_multi": (ctypes.c_int, [P, i32, P, P, f64, i32, i32, P, SPS]),
    "fvpcg_solve_mixed": (ctypes.c_int, [P, P, P, f64, f64, i32, i32, P, SPS]),
    "fvpcg_solve_mixed_reliable": (ctypes.c_int, [P, P, P, f64, i32, i32, P, SPS]),
    "fvpcg_solve_backward": (ctypes.c_int, [P, P, P, P, P, P, P, f64, i32, i32, i32, P, SPS]),
    "fvpcg_batch_create": (ctypes.c_int, [i32, P, P, P, P, P, P, P, u32, P, PP]),
    "fvpcg_batch_destroy": (ctypes.c_int, [P]),
    "fvpcg_solve_batched": (ctypes.c_int, [P, P, P, f64, i32, i32, i32, P, SPS]),
    "fvpcg_solve_batched_backward": (ctypes.c_int, [P, P, P, P, P, P, P, f64, i32, i32, i32, P, SPS]),
    "fvpcg_stream_calibrate": (ctypes.c_int, [P, u64, ctypes.POINTER(f64), ctypes.POINTER(f64)]),
    "fvpcg_stream_mix": (ctypes.c_int, [P, u64, i32, i32, ctypes.POINTER(f64)]),
    "fvpcg_assemble_transient": (ctypes.c_int, [P, P, P, P, P, P, f64, P, P, P, P, P]),
    "fvpcg_transient_run": (ctypes.c_int, [P, P, P, P, P, P, f64, i32, P, f64, i32, i32, P, SPS]),
    "fvpcg_amg_create": (ctypes.c_int, [P, f64, i32, i32, ctypes.c_uint64, P, PP]),
    "fvpcg_amg_export": (ctypes.c_int, [P, i32, i32, P, P, P, P, P, P]),
    "fvpcg_amg_refresh": (ctypes.c_int, [P, P]),
    "fvpcg_amg_destroy": (ctypes.c_int, [P]),
    "fvpcg_piso_create": (ctypes.c_int, [P, P, P, P, P, P, f64, f64, i32, P, PP]),
    "fvpcg_piso_destroy": (ctypes.c_int, [P]),
    "fvpcg_piso_run": (ctypes.c_int, [P, f64, i32, i32, P, P, P, f64, f64, i32, P, SPS]),
    "fvpcg_amg_info": (ctypes.c_int, [P, i32, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_int64)]),
    "fvpcg_amg_aggregates": (ctypes.c_int, [P, i32, P]),
    "fvpcg_amg_apply": (ctypes.c_int, [P, P, P, P]),
    "fvpcg_solve_amg": (ctypes.c_int, [P, P, P, f64, i32, i32, P, SPS]),
}

_lib = None


class ExtensionMissing(ImportError):
    pass


def load():
    """Load libfvpcg.so (raises ExtensionMissing if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  -- binds the library to torch's HIP runtime

    if not os.path.exists(LIB_PATH):
        raise ExtensionMissing(f"{LIB_PATH} is not built: run `python -m paper_1505_07630_amd.build` "
                               "(or __graft_entry__.build()) first; there is no fallback path")
    L = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L
