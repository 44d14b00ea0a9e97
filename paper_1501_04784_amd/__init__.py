"""MI355X-native builder of the lower-triangular Poisson stiffness matrix.

Python face of the C ABI in ``include/kbuild.h`` (``libkbuild.so``).  This module
only marshals arguments: device memory comes from torch, every step of the
integration and assembly runs in the library's HIP kernels on the current torch
stream.  There is no CPU path; a missing library raises ``ImportError``.

    from paper_1501_04784_amd import build_lower_csr
    K = build_lower_csr(conn, coords, coef, elem=8, prec="fp32fb64")   # device tensors
    K.row_ptr, K.col_idx, K.vals            # lower-triangular CSR, int32 indices
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import _lib
from ._lib import (KB_F_CAPACITY, KB_F_INDEX, KB_F_INVERTED, KB_F_NONFINITE, KB_F_REPEAT, KB_FP32, KB_FP32_FB64,
                   KB_FP64, KB_HEX8, KB_N_STAGES, KB_STATUS_WORDS, KB_TET4, STAGE_NAMES, KbMesh, KbTuning)

PRECISIONS = {"fp64": KB_FP64, "fp32": KB_FP32, "fp32fb64": KB_FP32_FB64}
FLAG_NAMES = {KB_F_INDEX: "index", KB_F_REPEAT: "repeat", KB_F_INVERTED: "inverted", KB_F_NONFINITE: "nonfinite",
              KB_F_CAPACITY: "capacity"}


class KBuildError(RuntimeError):
    pass


def status_string(code: int) -> str:
    return _lib.lib().kb_status_string(int(code)).decode()


def version() -> int:
    return int(_lib.lib().kb_version())


def _prec(prec) -> int:
    if isinstance(prec, str):
        return PRECISIONS[prec]
    if prec in (KB_FP64, KB_FP32, KB_FP32_FB64):
        return int(prec)
    raise ValueError(f"unknown precision {prec!r}")


def value_dtype(prec) -> torch.dtype:
    return torch.float64 if _prec(prec) == KB_FP64 else torch.float32


def _check(rc: int, what: str):
    if rc != 0:
        raise KBuildError(f"{what}: {status_string(rc)} ({rc})")


def _ptr(t: torch.Tensor | None):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _mesh(elem, n_elem, n_node, conn=None, coords=None, coef=None) -> KbMesh:
    return KbMesh(int(elem), 0, int(n_elem), int(n_node), None if conn is None else conn.data_ptr(),
                  None if coords is None else coords.data_ptr(), None if coef is None else coef.data_ptr())


@dataclass
class Tuning:
    block: int = 0
    bucket_bits: int = 0
    fb_tau: float = 0.0
    sub_bits: int = 0

    def to_c(self, events=None) -> KbTuning:
        return KbTuning(int(self.block), int(self.bucket_bits), float(self.fb_tau), int(self.sub_bits), events)


def plan(elem: int, n_elem: int, n_node: int, prec="fp64", tuning: Tuning | None = None):
    """(workspace bytes, number of triplets) for a mesh shape."""
    ws = ctypes.c_size_t(0)
    nt = ctypes.c_int64(0)
    m = _mesh(elem, n_elem, n_node)
    tu = (tuning or Tuning()).to_c()
    _check(_lib.lib().kb_plan(ctypes.byref(m), _prec(prec), ctypes.byref(tu), ctypes.byref(ws), ctypes.byref(nt)),
           "kb_plan")
    return int(ws.value), int(nt.value)


def _validate_mesh(conn, coords, coef, elem, need_geometry=True):
    if elem not in (KB_HEX8, KB_TET4):
        raise ValueError("elem must be 8 (hex8) or 4 (tet4)")
    if conn.dtype != torch.int32 or conn.dim() != 2 or conn.shape[1] != elem or not conn.is_contiguous():
        raise ValueError(f"conn must be a contiguous int32 [n_elem, {elem}] tensor")
    if not conn.is_cuda:
        raise ValueError("conn must be a device tensor")
    if need_geometry:
        if coords.dtype != torch.float64 or coords.dim() != 2 or coords.shape[1] != 3 or not coords.is_contiguous():
            raise ValueError("coords must be a contiguous float64 [n_node, 3] tensor")
        if coef.dtype != torch.float64 or coef.shape != (conn.shape[0],) or not coef.is_contiguous():
            raise ValueError("coef must be a contiguous float64 [n_elem] tensor")
        if not (coords.is_cuda and coef.is_cuda):
            raise ValueError("coords and coef must be device tensors")


@dataclass
class LowerCSR:
    """Lower-triangular CSR of K (device tensors) plus the device status words."""

    row_ptr: torch.Tensor
    col_idx: torch.Tensor
    vals: torch.Tensor
    nnz: int
    status: torch.Tensor  # uint32-as-int32 [KB_STATUS_WORDS]

    @property
    def flags(self) -> int:
        return int(self.status[0].item()) & 0xFFFFFFFF

    @property
    def n_fallback(self) -> int:
        return int(self.status[1].item()) & 0xFFFFFFFF

    def to_torch(self) -> torch.Tensor:
        n = self.row_ptr.numel() - 1
        return torch.sparse_csr_tensor(self.row_ptr, self.col_idx, self.vals, size=(n, n))


def _raise_on_flags(flags: int, allow: int = 0):
    bad = flags & ~allow
    if bad:
        names = [v for k, v in FLAG_NAMES.items() if bad & k]
        raise KBuildError(f"data errors: {', '.join(names)} (flags={bad:#x})")


class Builder:
    """Reusable build context: workspace and outputs are allocated once per mesh shape.

    ``run`` enqueues one full construction on the current stream and allocates nothing,
    so repeated builds (and the benchmark's timed loop) only launch kernels.
    """

    def __init__(self, elem: int, n_elem: int, n_node: int, prec="fp32fb64", tuning: Tuning | None = None,
                 device="cuda", cap: int | None = None):
        self.elem, self.n_elem, self.n_node = int(elem), int(n_elem), int(n_node)
        self.prec = _prec(prec)
        self.tuning = tuning or Tuning()
        self.ws_bytes, self.n_triplets = plan(elem, n_elem, n_node, self.prec, self.tuning)
        self.cap = self.n_triplets if cap is None else int(cap)
        dev = torch.device(device)
        self.ws = torch.empty(max(self.ws_bytes, 1), dtype=torch.uint8, device=dev)
        self.row_ptr = torch.empty(self.n_node + 1, dtype=torch.int32, device=dev)
        self.col_idx = torch.empty(max(self.cap, 1), dtype=torch.int32, device=dev)
        self.vals = torch.empty(max(self.cap, 1), dtype=value_dtype(self.prec), device=dev)
        self.nnz_dev = torch.zeros(1, dtype=torch.int64, device=dev)
        self.status = torch.zeros(KB_STATUS_WORDS, dtype=torch.int32, device=dev)

    def run(self, conn, coords, coef, stage_events=None, stream=None, klow=None):
        """Enqueue the construction (or assembly only, if ``klow`` is given)."""
        s = stream if stream is not None else torch.cuda.current_stream()
        ev = None
        if stage_events is not None:
            arr = (ctypes.c_void_p * len(stage_events))(*[int(e) for e in stage_events])
            self._ev_keep = arr
            ev = ctypes.cast(arr, ctypes.c_void_p)
        tu = self.tuning.to_c(ev)
        m = _mesh(self.elem, self.n_elem, self.n_node, conn, coords, coef)
        L = _lib.lib()
        if klow is None:
            rc = L.kb_build_lower_csr(ctypes.byref(m), self.prec, ctypes.byref(tu), _ptr(self.ws), self.ws_bytes,
                                      _ptr(self.row_ptr), _ptr(self.col_idx), _ptr(self.vals), self.cap,
                                      _ptr(self.nnz_dev), _ptr(self.status), ctypes.c_void_p(s.cuda_stream))
            _check(rc, "kb_build_lower_csr")
        else:
            rc = L.kb_assemble_lower_csr(ctypes.byref(m), self.prec, ctypes.byref(tu), _ptr(klow), _ptr(self.ws),
                                         self.ws_bytes, _ptr(self.row_ptr), _ptr(self.col_idx), _ptr(self.vals),
                                         self.cap, _ptr(self.nnz_dev), _ptr(self.status),
                                         ctypes.c_void_p(s.cuda_stream))
            _check(rc, "kb_assemble_lower_csr")

    def result(self, check: bool = True, allow_flags: int = 0) -> LowerCSR:
        """Synchronise and return the (trimmed) CSR; raise on data errors if ``check``."""
        torch.cuda.current_stream().synchronize()
        nnz = int(self.nnz_dev.item())
        st = self.status.clone()
        res = LowerCSR(self.row_ptr, self.col_idx[:nnz] if nnz <= self.cap else self.col_idx[:0],
                       self.vals[:nnz] if nnz <= self.cap else self.vals[:0], nnz, st)
        if check:
            _raise_on_flags(res.flags, allow_flags)
        return res


def build_lower_csr(conn, coords, coef, elem: int, prec="fp32fb64", tuning: Tuning | None = None, check=True,
                    allow_flags: int = 0, cap: int | None = None) -> LowerCSR:
    """Integrate and assemble lower-triangular CSR K on the GPU (one call)."""
    _validate_mesh(conn, coords, coef, elem)
    b = Builder(elem, conn.shape[0], coords.shape[0], prec, tuning, device=conn.device, cap=cap)
    b.run(conn, coords, coef)
    return b.result(check=check, allow_flags=allow_flags)


def assemble_lower_csr(conn, n_node: int, klow, elem: int, prec="fp64", tuning: Tuning | None = None, check=True,
                       allow_flags: int = 0, cap: int | None = None) -> LowerCSR:
    """Assemble lower CSR K from given per-element lower values klow [n_elem, nen(nen+1)/2]."""
    _validate_mesh(conn, None, None, elem, need_geometry=False)
    te = elem * (elem + 1) // 2
    if klow.dtype != value_dtype(prec) or klow.shape != (conn.shape[0], te) or not klow.is_contiguous():
        raise ValueError(f"klow must be a contiguous {value_dtype(prec)} [n_elem, {te}] tensor")
    b = Builder(elem, conn.shape[0], n_node, prec, tuning, device=conn.device, cap=cap)
    b.run(conn, None, None, klow=klow)
    return b.result(check=check, allow_flags=allow_flags)


def integrate_lower(conn, coords, coef, elem: int, prec="fp64", tuning: Tuning | None = None, check=True,
                    allow_flags: int = 0):
    """Per-element packed lower triangles [n_elem, nen(nen+1)/2] (Alg. 2 only)."""
    _validate_mesh(conn, coords, coef, elem)
    te = elem * (elem + 1) // 2
    out = torch.empty((conn.shape[0], te), dtype=value_dtype(prec), device=conn.device)
    status = torch.zeros(KB_STATUS_WORDS, dtype=torch.int32, device=conn.device)
    m = _mesh(elem, conn.shape[0], coords.shape[0], conn, coords, coef)
    tu = (tuning or Tuning()).to_c()
    rc = _lib.lib().kb_integrate_lower(ctypes.byref(m), _prec(prec), ctypes.byref(tu), _ptr(out), _ptr(status),
                                       ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    _check(rc, "kb_integrate_lower")
    torch.cuda.current_stream().synchronize()
    flags = int(status[0].item()) & 0xFFFFFFFF
    if check:
        _raise_on_flags(flags, allow_flags)
    return out, status


__all__ = ["Builder", "LowerCSR", "KBuildError", "Tuning", "build_lower_csr", "assemble_lower_csr",
           "integrate_lower", "plan", "status_string", "version", "value_dtype", "STAGE_NAMES", "KB_N_STAGES",
           "KB_HEX8", "KB_TET4", "KB_FP64", "KB_FP32", "KB_FP32_FB64"]
