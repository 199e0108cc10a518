"""ctypes declarations of libvqe.so (the C ABI in include/vqe.h).

Loads the in-tree library only.  There is no fallback: if libvqe.so is not
built, every use raises.
"""
from __future__ import annotations

import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvqe.so")

VQE_OK = 0
VQE_EINVAL = -1
VQE_ENOMEM = -2
VQE_EUNSUPPORTED = -3
VQE_EHIP = -4
NOALLOC_SCRATCH_BYTES = 8 << 20  # VQE_NOALLOC_SCRATCH_BYTES

GATE_CODES = {
    "RX": 0, "RY": 1, "RZ": 2, "H": 3, "X": 4,
    "CNOT": 5, "CZ": 6, "SingleExcitation": 7, "DoubleExcitation": 8,
}
OPT_ADAM = 0
OPT_GD = 1

EXPORTED = [
    "vqe_ctx_create", "vqe_ctx_destroy", "vqe_ctx_set_mem_budget", "vqe_ctx_set_tile",
    "vqe_ctx_reserve", "vqe_ctx_set_loop_mode", "vqe_ctx_set_staged", "vqe_last_error", "vqe_strerror",
    "vqe_ham_create", "vqe_ham_from_integrals", "vqe_ham_info", "vqe_ham_terms", "vqe_ham_destroy",
    "vqe_circ_create", "vqe_circ_destroy", "vqe_workspace_bytes",
    "vqe_prepare_reference", "vqe_apply_ansatz", "vqe_expect", "vqe_energy",
    "vqe_apply_hamiltonian", "vqe_energy_grad", "vqe_grad_shift", "vqe_adam_step", "vqe_run",
    "vqe_circ_plan_export", "vqe_ham_plan_export",
    "vqe_hfam_create", "vqe_hfam_info", "vqe_hfam_member", "vqe_hfam_set_integrals", "vqe_hfam_destroy",
    "vqe_ctx_set_profiling", "vqe_ctx_profile", "vqe_stream_create", "vqe_stream_destroy",
    "vqe_apply_ansatz_noalloc", "vqe_ctx_set_graphs", "vqe_ctx_graph_stats", "vqe_ctx_clear_tuning",
    "vqe_autotune", "vqe_tune_set",
]


class KernelStat(ctypes.Structure):
    """vqe_kernel_stat."""
    _fields_ = [("name", ctypes.c_char * 48), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double),
                ("bytes", ctypes.c_double)]


class TuneResult(ctypes.Structure):
    """vqe_tune_result."""
    _fields_ = [("k_fwd", ctypes.c_int), ("k_rev", ctypes.c_int), ("c_low", ctypes.c_int), ("wg_max", ctypes.c_int),
                ("batch_tile", ctypes.c_int64), ("ms_default", ctypes.c_double), ("ms_tuned", ctypes.c_double),
                ("candidates", ctypes.c_int)]


class VQEError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"{message} [{code}]")
        self.code = code


class LibraryMissing(ImportError):
    pass


_lock = threading.Lock()
_lib = None


def _declare(L):
    P = ctypes.c_void_p
    i32, i64, u64, f64, sz = ctypes.c_int, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double, ctypes.c_size_t
    PP = ctypes.POINTER(ctypes.c_void_p)
    sig = {
        "vqe_ctx_create": [i32, PP],
        "vqe_ctx_destroy": [P],
        "vqe_ctx_set_mem_budget": [P, sz],
        "vqe_ctx_set_tile": [P, i32, i32, i32],
        "vqe_ctx_reserve": [P, sz],
        "vqe_ctx_set_loop_mode": [P, i32],
        "vqe_ctx_set_staged": [P, i32],
        "vqe_ham_create": [P, i32, i64, P, P, P, PP],
        "vqe_ham_from_integrals": [P, i32, P, P, f64, PP],
        "vqe_ham_info": [P, P, P, P],
        "vqe_ham_terms": [P, P, P, P],
        "vqe_ham_destroy": [P],
        "vqe_circ_create": [P, i32, i64, P, P, P, P, i32, PP],
        "vqe_circ_destroy": [P],
        "vqe_workspace_bytes": [P, P, i32, P, i64, i32, ctypes.POINTER(sz)],
        "vqe_prepare_reference": [P, i32, i64, u64, P, P],
        "vqe_apply_ansatz": [P, P, i64, P, P, P],
        "vqe_expect": [P, i32, P, i64, P, P, P],
        "vqe_apply_hamiltonian": [P, i32, P, i64, P, P, P],
        "vqe_energy": [P, P, i32, P, i64, u64, P, P, P, sz, P],
        "vqe_energy_grad": [P, P, i32, P, i64, u64, P, P, P, P, sz, P],
        "vqe_grad_shift": [P, P, i32, P, i64, u64, P, P, P, P, sz, P],
        "vqe_adam_step": [P, i64, i32, P, P, P, P, i32, f64, f64, f64, f64, P],
        "vqe_run": [P, P, i32, P, i64, u64, P, i32, i32, f64, f64, f64, f64, P, P, sz, P],
        "vqe_circ_plan_export": [P, P, i32, P, sz, ctypes.POINTER(sz)],
        "vqe_ham_plan_export": [P, i32, P, i64, i32, P, sz, ctypes.POINTER(sz)],
        "vqe_hfam_create": [P, i32, i64, PP],
        "vqe_hfam_info": [P, P, P, P],
        "vqe_hfam_member": [P, i64, PP],
        "vqe_hfam_set_integrals": [P, P, i64, i64, P, P],
        "vqe_hfam_destroy": [P],
        "vqe_ctx_set_profiling": [P, i32],
        "vqe_ctx_profile": [P, P, i32, P, i32],
        "vqe_stream_create": [P, PP],
        "vqe_stream_destroy": [P, P],
        "vqe_apply_ansatz_noalloc": [P, P, i64, P, P, P],
        "vqe_ctx_set_graphs": [P, i32],
        "vqe_ctx_graph_stats": [P, P, P, P],
        "vqe_ctx_clear_tuning": [P],
        "vqe_autotune": [P, P, i32, P, i64, u64, i32, P, P, P],
        "vqe_tune_set": [P, P, i64, i32, P],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = i32
    L.vqe_last_error.argtypes = [P]
    L.vqe_last_error.restype = ctypes.c_char_p
    L.vqe_strerror.argtypes = [i32]
    L.vqe_strerror.restype = ctypes.c_char_p


def lib():
    """The loaded libvqe.so (raises LibraryMissing if it has not been built)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise LibraryMissing(
                    f"{LIB_PATH} is not built; run `python -c 'import __graft_entry__ as g; g.build()'` "
                    "or `python paper_2601_09951_amd/build.py`")
            L = ctypes.CDLL(LIB_PATH)
            _declare(L)
            _lib = L
    return _lib


def check(rc: int, ctx=None) -> None:
    if rc != VQE_OK:
        L = lib()
        msg = L.vqe_last_error(ctx).decode() if ctx else ""
        raise VQEError(rc, f"{L.vqe_strerror(rc).decode()}: {msg}")
