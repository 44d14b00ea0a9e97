"""ctypes binding of ``libkbuild.so`` (argument marshalling only; no compute here)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkbuild.so")

KB_HEX8, KB_TET4 = 8, 4
KB_OP_STIFFNESS, KB_OP_MASS = 0, 1
KB_FP64, KB_FP32, KB_FP32_FB64 = 0, 1, 2
KB_OK, KB_EINVAL, KB_ERANGE, KB_ENOSPC, KB_EHIP = 0, -1, -2, -3, -4
KB_STATUS_WORDS = 4
KB_F_INDEX, KB_F_REPEAT, KB_F_INVERTED, KB_F_NONFINITE, KB_F_CAPACITY = 1, 2, 4, 8, 16
KB_N_STAGES = 8
KB_SCRATCH_BYTES = 64 << 20  # fixed workspace of kb_build_lower_csr_noalloc
STAGE_NAMES = ("init", "count", "offsets", "integrate", "histogram", "partition", "reduce", "compress")

# every function declared in include/kbuild.h
EXPORTS = ("kb_plan", "kb_build_lower_csr", "kb_build_lower_csr_noalloc", "kb_integrate_lower", "kb_assemble_lower_csr", "kb_plan_dof",
           "kb_assemble_lower_csr_dof", "kb_plan_grouped", "kb_build_lower_csr_grouped",
           "kb_build_lower_csr_group_pass", "kb_plan_batched", "kb_build_lower_csr_batched", "kb_plan_adjoint",
           "kb_adjoint_lower", "kb_status_string", "kb_version")


class KbMesh(ctypes.Structure):
    _fields_ = [
        ("elem", ctypes.c_int32),
        ("op", ctypes.c_int32),
        ("n_elem", ctypes.c_int64),
        ("n_node", ctypes.c_int64),
        ("conn", ctypes.c_void_p),
        ("coords", ctypes.c_void_p),
        ("coef", ctypes.c_void_p),
    ]


class KbBatch(ctypes.Structure):
    _fields_ = [
        ("elem", ctypes.c_int32),
        ("n_mesh", ctypes.c_int32),
        ("n_elem", ctypes.c_int64),
        ("n_node", ctypes.c_int64),
        ("elem_off", ctypes.c_void_p),
        ("node_off", ctypes.c_void_p),
        ("conn", ctypes.c_void_p),
        ("coords", ctypes.c_void_p),
        ("coef", ctypes.c_void_p),
    ]


class KbTuning(ctypes.Structure):
    _fields_ = [
        ("block", ctypes.c_int32),
        ("bucket_bits", ctypes.c_int32),
        ("fb_tau", ctypes.c_float),
        ("sub_bits", ctypes.c_int32),
        ("stage_events", ctypes.c_void_p),
        ("seg_pairs", ctypes.c_int32),
        ("table_slots", ctypes.c_int32),
    ]


_lib = None


def lib():
    """Load the HIP library; raise if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'` "
                "or `python paper_1501_04784_amd/build.py`")
        L = ctypes.CDLL(LIB_PATH)
        p, i32, i64, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_size_t
        PM, PT = ctypes.POINTER(KbMesh), ctypes.POINTER(KbTuning)
        L.kb_plan.argtypes = [PM, i32, PT, ctypes.POINTER(sz), ctypes.POINTER(i64)]
        L.kb_plan.restype = i32
        L.kb_build_lower_csr.argtypes = [PM, i32, PT, p, sz, p, p, p, i64, p, p, p]
        L.kb_build_lower_csr.restype = i32
        L.kb_build_lower_csr_noalloc.argtypes = [PM, i32, PT, p, p, p, i64, p, p, p]
        L.kb_build_lower_csr_noalloc.restype = i32
        L.kb_integrate_lower.argtypes = [PM, i32, PT, p, p, p]
        L.kb_integrate_lower.restype = i32
        L.kb_assemble_lower_csr.argtypes = [PM, i32, PT, p, p, sz, p, p, p, i64, p, p, p]
        L.kb_assemble_lower_csr.restype = i32
        L.kb_plan_dof.argtypes = [PM, i32, i32, PT, ctypes.POINTER(sz), ctypes.POINTER(i64)]
        L.kb_plan_dof.restype = i32
        L.kb_assemble_lower_csr_dof.argtypes = [PM, i32, i32, PT, p, p, sz, p, p, p, i64, p, p, p]
        L.kb_assemble_lower_csr_dof.restype = i32
        L.kb_plan_grouped.argtypes = [PM, i32, PT, i64, i64, ctypes.POINTER(sz)]
        L.kb_plan_grouped.restype = i32
        L.kb_build_lower_csr_grouped.argtypes = [PM, i32, PT, i64, p, sz, p, p, p, i64, p, p, p]
        L.kb_build_lower_csr_grouped.restype = i32
        L.kb_build_lower_csr_group_pass.argtypes = [PM, i32, PT, i64, i64, p, p, p, sz, p, p, p, i64, p, p, p]
        L.kb_build_lower_csr_group_pass.restype = i32
        PB = ctypes.POINTER(KbBatch)
        L.kb_plan_batched.argtypes = [PB, i32, PT, ctypes.POINTER(sz), ctypes.POINTER(i64)]
        L.kb_plan_batched.restype = i32
        L.kb_build_lower_csr_batched.argtypes = [PB, i32, PT, p, sz, p, p, p, i64, p, p, p]
        L.kb_build_lower_csr_batched.restype = i32
        L.kb_plan_adjoint.argtypes = [PM, ctypes.POINTER(sz)]
        L.kb_plan_adjoint.restype = i32
        L.kb_adjoint_lower.argtypes = [PM, p, p, p, i64, p, sz, p, p, p, p]
        L.kb_adjoint_lower.restype = i32
        L.kb_status_string.argtypes = [i32]
        L.kb_status_string.restype = ctypes.c_char_p
        L.kb_version.argtypes = []
        L.kb_version.restype = i32
        _lib = L
    return _lib


# ---- HIP events (same runtime instance as the library and torch) --------------------
class HipEvents:
    """A set of HIP timing events, resolved through the library's own HIP runtime."""

    def __init__(self, n: int):
        L = lib()
        self._L = L
        L.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        L.hipEventCreate.restype = ctypes.c_int
        L.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p]
        L.hipEventElapsedTime.restype = ctypes.c_int
        L.hipEventDestroy.argtypes = [ctypes.c_void_p]
        L.hipEventDestroy.restype = ctypes.c_int
        self.handles = []
        for _ in range(n):
            h = ctypes.c_void_p()
            if L.hipEventCreate(ctypes.byref(h)) != 0:
                raise RuntimeError("hipEventCreate failed")
            self.handles.append(h.value)

    def elapsed_ms(self, i: int, j: int) -> float:
        ms = ctypes.c_float(0.0)
        if self._L.hipEventElapsedTime(ctypes.byref(ms), self.handles[i], self.handles[j]) != 0:
            raise RuntimeError("hipEventElapsedTime failed")
        return float(ms.value)

    def close(self):
        for h in self.handles:
            self._L.hipEventDestroy(h)
        self.handles = []
