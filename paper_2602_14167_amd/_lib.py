"""ctypes binding of libtcng.so (argument marshalling only).

Every step of the computation runs in the HIP kernels behind the C ABI in
include/tcng.h.  There is no CPU fallback: if the library is missing or no
HIP device is present, the calls raise.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtcng.so")

TCNG_OK, TCNG_E_INVALID, TCNG_E_UNSUPPORTED, TCNG_E_WORKSPACE, TCNG_E_HIP, TCNG_E_ALLOC = range(6)
TCNG_C64, TCNG_C128 = 0, 1
TCNG_MODE_TILED, TCNG_MODE_PLAIN, TCNG_MODE_FUSED, TCNG_MODE_FUSED5, TCNG_MODE_AUTO = 0, 1, 2, 3, 4
TCNG_U1_KIND = 12   # constant one-qubit gate (top-left 2 x 2 block of its matrix)

# every function include/tcng.h declares
EXPORTS = [
    "tcng_last_error", "tcng_version", "tcng_state_init", "tcng_apply_gate", "tcng_circuit_create",
    "tcng_circuit_destroy", "tcng_circuit_num_passes", "tcng_pauli_sum_create", "tcng_pauli_sum_destroy",
    "tcng_workspace_size", "tcng_run_circuit", "tcng_expect_pauli", "tcng_expect_grad", "tcng_plan_inspect",
    "tcng_fused_plan_inspect", "tcng_rounds_plan_inspect", "tcng_graph_create", "tcng_graph_launch", "tcng_graph_destroy",
    "tcng_profile_begin", "tcng_profile_query", "tcng_profile_end", "tcng_circuit_configure",
    "tcng_circuit_get_config", "tcng_autotune", "tcng_workspace_size_multi", "tcng_expect_grad_multi",
    "tcng_mipt_workspace_size", "tcng_mipt_run", "tcng_apply_pauli", "tcng_pauli_coo_info", "tcng_pauli_coo",
    "tcng_shadow_workspace_size", "tcng_shadow_snapshots", "tcng_qml_workspace_size", "tcng_qml_step",
    "tcng_expect_grad_noalloc", "tcng_noalloc_scratch_bytes", "tcng_circuit_get_mode", "tcng_circuit_rounds",
    "tcng_multi_create",
    "tcng_multi_launch", "tcng_multi_destroy", "tcng_graph_create_multi",
]


class TcngState(ctypes.Structure):
    _fields_ = [("amps", ctypes.c_void_p), ("n_qubits", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("batch", ctypes.c_int64), ("stride", ctypes.c_int64)]


class TcngGate(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("q0", ctypes.c_int32), ("q1", ctypes.c_int32),
                ("p0", ctypes.c_int32), ("p1", ctypes.c_int32), ("mat", ctypes.c_int32)]


class TcngError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"tcng error {status}: {msg}")
        self.status = status


_lib = None


def lib():
    """Load libtcng.so (built in-tree by paper_2602_14167_amd/build.py)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing (run __graft_entry__.build())")
    L = ctypes.CDLL(LIB_PATH)
    P, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    PS = ctypes.POINTER(TcngState)
    L.tcng_last_error.restype = ctypes.c_char_p
    L.tcng_last_error.argtypes = []
    L.tcng_version.restype = i32
    L.tcng_state_init.argtypes = [PS, P, i64, P]
    L.tcng_apply_gate.argtypes = [PS, P, i32, P, P]
    L.tcng_circuit_create.argtypes = [i32, P, i32, i32, P, i32, ctypes.POINTER(P)]
    L.tcng_circuit_destroy.argtypes = [P]
    L.tcng_circuit_num_passes.argtypes = [P, i32, ctypes.POINTER(i32)]
    L.tcng_pauli_sum_create.argtypes = [i32, P, P, i32, ctypes.POINTER(P)]
    L.tcng_pauli_sum_destroy.argtypes = [P]
    L.tcng_workspace_size.argtypes = [P, P, i32, i64, i32, ctypes.POINTER(sz)]
    L.tcng_run_circuit.argtypes = [P, P, PS, i32, P, sz, P]
    L.tcng_expect_pauli.argtypes = [PS, P, P, i32, P, sz, P]
    L.tcng_expect_grad.argtypes = [P, P, P, PS, PS, P, P, P, i32, P, sz, P]
    L.tcng_expect_grad_noalloc.argtypes = [P, P, P, PS, PS, P, P, P, i32, P]
    L.tcng_noalloc_scratch_bytes.argtypes = []
    L.tcng_workspace_size_multi.argtypes = [P, P, i32, i32, ctypes.POINTER(sz)]
    L.tcng_expect_grad_multi.argtypes = [P, P, i32, P, PS, PS, P, P, P, P, sz, P]
    L.tcng_multi_create.argtypes = [P, P, i32, P, PS, PS, P, P, P, i64, P, sz, ctypes.POINTER(P)]
    L.tcng_multi_launch.argtypes = [P, P]
    L.tcng_multi_destroy.argtypes = [P]
    L.tcng_graph_create_multi.argtypes = [P, ctypes.POINTER(P)]
    L.tcng_circuit_configure.argtypes = [P, i32, i32, i32, i32]
    L.tcng_circuit_get_config.argtypes = [P, i32, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32)]
    L.tcng_circuit_get_mode.argtypes = [P, i32, ctypes.POINTER(i32)]
    L.tcng_circuit_rounds.argtypes = [P, i32, ctypes.POINTER(i32)]
    L.tcng_autotune.argtypes = [P, P, P, PS, PS, i32, ctypes.c_char_p, ctypes.POINTER(ctypes.c_double), P]
    L.tcng_profile_begin.argtypes = [i32]
    L.tcng_profile_query.argtypes = [i32, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double)]
    L.tcng_profile_end.argtypes = []
    L.tcng_plan_inspect.argtypes = [i32, P, i32, i32, i32, P, P, P, ctypes.POINTER(i32)]
    L.tcng_graph_create.argtypes = [P, P, P, PS, PS, P, P, P, i32, P, sz, i64, ctypes.POINTER(P)]
    L.tcng_graph_launch.argtypes = [P, P]
    L.tcng_graph_destroy.argtypes = [P]
    L.tcng_fused_plan_inspect.argtypes = [i32, P, i32, i32, i32, P, P, P, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                          ctypes.POINTER(i32)]
    L.tcng_rounds_plan_inspect.argtypes = [i32, P, i32, i32, i32, i32, i32, ctypes.POINTER(i32),
                                           ctypes.POINTER(i32), ctypes.POINTER(i32)]
    L.tcng_apply_pauli.argtypes = [PS, P, PS, P, i32, P, sz, P]
    L.tcng_pauli_coo_info.argtypes = [P, ctypes.POINTER(i32)]
    L.tcng_pauli_coo.argtypes = [P, i64, i64, P, P, P, P]
    L.tcng_qml_workspace_size.argtypes = [P, i64, ctypes.POINTER(sz)]
    L.tcng_qml_step.argtypes = [P, P, PS, PS, PS, P, i32, i32, P, P, P, sz, P]
    L.tcng_shadow_workspace_size.argtypes = [P, i64, ctypes.POINTER(sz)]
    L.tcng_shadow_snapshots.argtypes = [P, P, PS, P, P, P, P, sz, P]
    L.tcng_mipt_workspace_size.argtypes = [P, i32, i64, ctypes.POINTER(sz)]
    L.tcng_mipt_run.argtypes = [P, i32, P, PS, P, ctypes.c_double, P, P, P, P, sz, P]
    for name in EXPORTS:
        if name not in ("tcng_last_error", "tcng_version", "tcng_noalloc_scratch_bytes"):
            getattr(L, name).restype = i32
    L.tcng_noalloc_scratch_bytes.restype = sz
    _lib = L
    return L


def check(status):
    if status != TCNG_OK:
        msg = lib().tcng_last_error().decode(errors="replace")
        raise TcngError(status, msg)
