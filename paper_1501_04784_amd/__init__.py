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
                   KB_FP64, KB_HEX8, KB_N_STAGES, KB_OP_MASS, KB_OP_STIFFNESS, KB_STATUS_WORDS, KB_TET4, STAGE_NAMES,
                   KbBatch, KbMesh, KbTuning)

PRECISIONS = {"fp64": KB_FP64, "fp32": KB_FP32, "fp32fb64": KB_FP32_FB64}
OPERATORS = {"stiffness": KB_OP_STIFFNESS, "mass": KB_OP_MASS}
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


def _op(op) -> int:
    if isinstance(op, str):
        return OPERATORS[op]
    if op in (KB_OP_STIFFNESS, KB_OP_MASS):
        return int(op)
    raise ValueError(f"unknown operator {op!r}")


def _mesh(elem, n_elem, n_node, conn=None, coords=None, coef=None, op="stiffness") -> KbMesh:
    return KbMesh(int(elem), _op(op), int(n_elem), int(n_node), None if conn is None else conn.data_ptr(),
                  None if coords is None else coords.data_ptr(), None if coef is None else coef.data_ptr())


@dataclass(frozen=True)
class Tuning:
    block: int = 0
    bucket_bits: int = 0
    fb_tau: float = 0.0
    sub_bits: int = 0
    seg_pairs: int = 0
    table_slots: int = 0

    def to_c(self, events=None) -> KbTuning:
        return KbTuning(int(self.block), int(self.bucket_bits), float(self.fb_tau), int(self.sub_bits), events,
                        int(self.seg_pairs), int(self.table_slots))


def plan(elem: int, n_elem: int, n_node: int, prec="fp64", tuning: Tuning | None = None, op="stiffness",
         dof: int = 1):
    """(workspace bytes, number of triplets) for a mesh shape (``dof`` > 1: assembly of
    element matrices with that many components per node)."""
    ws = ctypes.c_size_t(0)
    nt = ctypes.c_int64(0)
    m = _mesh(elem, n_elem, n_node, op=op)
    tu = (tuning or Tuning()).to_c()
    if dof == 1:
        rc = _lib.lib().kb_plan(ctypes.byref(m), _prec(prec), ctypes.byref(tu), ctypes.byref(ws), ctypes.byref(nt))
        _check(rc, "kb_plan")
    else:
        rc = _lib.lib().kb_plan_dof(ctypes.byref(m), int(dof), _prec(prec), ctypes.byref(tu), ctypes.byref(ws),
                                    ctypes.byref(nt))
        _check(rc, "kb_plan_dof")
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
        """The matrix as ``torch.sparse_csr_tensor`` (int32 indices), sharing this CSR's memory."""
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
                 device="cuda", cap: int | None = None, op="stiffness", dof: int = 1):
        self.elem, self.n_elem, self.n_node = int(elem), int(n_elem), int(n_node)
        self.prec = _prec(prec)
        self.op = _op(op)
        self.dof = int(dof)
        self.tuning = tuning or Tuning()
        self.ws_bytes, self.n_triplets = plan(elem, n_elem, n_node, self.prec, self.tuning, self.op, self.dof)
        self.cap = self.n_triplets if cap is None else int(cap)
        dev = torch.device(device)
        self.ws = torch.empty(max(self.ws_bytes, 1), dtype=torch.uint8, device=dev)
        self.row_ptr = torch.empty(self.dof * self.n_node + 1, dtype=torch.int32, device=dev)
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
        m = _mesh(self.elem, self.n_elem, self.n_node, conn, coords, coef, self.op)
        L = _lib.lib()
        if self.dof != 1:
            if klow is None:
                raise ValueError("several DOFs per node: element values klow are required")
            rc = L.kb_assemble_lower_csr_dof(ctypes.byref(m), self.dof, self.prec, ctypes.byref(tu), _ptr(klow),
                                             _ptr(self.ws), self.ws_bytes, _ptr(self.row_ptr), _ptr(self.col_idx),
                                             _ptr(self.vals), self.cap, _ptr(self.nnz_dev), _ptr(self.status),
                                             ctypes.c_void_p(s.cuda_stream))
            _check(rc, "kb_assemble_lower_csr_dof")
        elif klow is None:
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
                    allow_flags: int = 0, cap: int | None = None, op="stiffness") -> LowerCSR:
    """Integrate and assemble lower-triangular CSR K (or the consistent mass matrix with
    op="mass") on the GPU (one call)."""
    _validate_mesh(conn, coords, coef, elem)
    b = Builder(elem, conn.shape[0], coords.shape[0], prec, tuning, device=conn.device, cap=cap, op=op)
    b.run(conn, coords, coef)
    return b.result(check=check, allow_flags=allow_flags)


def lower_csr_tensor(conn, coords, coef, elem: int, prec="fp32fb64", tuning: Tuning | None = None,
                     op="stiffness") -> torch.Tensor:
    """Lower-triangular K as a ``torch.sparse_csr_tensor`` (int32 indices, trimmed to nnz,
    values float64 for "fp64", float32 otherwise) on the mesh's device; raises
    ``KBuildError`` on data errors."""
    return build_lower_csr(conn, coords, coef, elem, prec=prec, tuning=tuning, op=op).to_torch()


def build_lower_csr_noalloc(conn, coords, coef, elem: int, row_ptr, col_idx, vals, nnz_dev, status, prec="fp32fb64",
                            tuning: Tuning | None = None, op="stiffness", stream=None):
    """Enqueue a full construction into caller-allocated outputs through
    ``kb_build_lower_csr_noalloc``: the library's fixed per-device scratch replaces the
    workspace, and nothing is allocated (outputs as for ``Builder``; the mesh's workspace
    must fit ``KB_SCRATCH_BYTES``).  Calls on one device must not overlap."""
    _validate_mesh(conn, coords, coef, elem)
    s = stream if stream is not None else torch.cuda.current_stream()
    tu = (tuning or Tuning()).to_c()
    m = _mesh(elem, conn.shape[0], coords.shape[0], conn, coords, coef, op)
    rc = _lib.lib().kb_build_lower_csr_noalloc(ctypes.byref(m), _prec(prec), ctypes.byref(tu), _ptr(row_ptr),
                                               _ptr(col_idx), _ptr(vals), int(col_idx.numel()), _ptr(nnz_dev),
                                               _ptr(status), ctypes.c_void_p(s.cuda_stream))
    _check(rc, "kb_build_lower_csr_noalloc")


def assemble_lower_csr(conn, n_node: int, klow, elem: int, prec="fp64", tuning: Tuning | None = None, check=True,
                       allow_flags: int = 0, cap: int | None = None, dof: int = 1) -> LowerCSR:
    """Assemble lower CSR K from given per-element lower values klow [n_elem, nd(nd+1)/2],
    nd = elem * dof (local row a * dof + i is component i of corner a; K has dof * n_node
    rows)."""
    _validate_mesh(conn, None, None, elem, need_geometry=False)
    nd = elem * int(dof)
    te = nd * (nd + 1) // 2
    if klow.dtype != value_dtype(prec) or klow.shape != (conn.shape[0], te) or not klow.is_contiguous():
        raise ValueError(f"klow must be a contiguous {value_dtype(prec)} [n_elem, {te}] tensor")
    b = Builder(elem, conn.shape[0], n_node, prec, tuning, device=conn.device, cap=cap, dof=dof)
    b.run(conn, None, None, klow=klow)
    return b.result(check=check, allow_flags=allow_flags)


# ---- grouped builds (Eq. 10) -------------------------------------------------------------
def plan_grouped(elem: int, n_elem: int, n_node: int, group_elems: int, cap: int, prec="fp32fb64",
                 tuning: Tuning | None = None, op="stiffness") -> int:
    """Workspace bytes of a grouped build."""
    ws = ctypes.c_size_t(0)
    m = _mesh(elem, n_elem, n_node, op=op)
    tu = (tuning or Tuning()).to_c()
    _check(_lib.lib().kb_plan_grouped(ctypes.byref(m), _prec(prec), ctypes.byref(tu), int(group_elems), int(cap),
                                      ctypes.byref(ws)), "kb_plan_grouped")
    return int(ws.value)


class GroupedBuilder:
    """Reusable grouped build (elements in groups of ``group_elems``, one pass each;
    ``cap`` bounds the final nnz).  ``run`` enqueues the passes and allocates nothing."""

    def __init__(self, elem: int, n_elem: int, n_node: int, group_elems: int, cap: int, prec="fp32fb64",
                 tuning: Tuning | None = None, device="cuda", op="stiffness"):
        self.elem, self.n_elem, self.n_node = int(elem), int(n_elem), int(n_node)
        self.group, self.cap = int(group_elems), int(cap)
        self.prec, self.op = _prec(prec), _op(op)
        self.tuning = tuning or Tuning()
        self.ws_bytes = plan_grouped(elem, n_elem, n_node, self.group, self.cap, self.prec, self.tuning, self.op)
        dev = torch.device(device)
        self.ws = torch.empty(max(self.ws_bytes, 1), dtype=torch.uint8, device=dev)
        self.row_ptr = torch.empty(self.n_node + 1, dtype=torch.int32, device=dev)
        self.col_idx = torch.empty(max(self.cap, 1), dtype=torch.int32, device=dev)
        self.vals = torch.empty(max(self.cap, 1), dtype=value_dtype(self.prec), device=dev)
        self.nnz_dev = torch.zeros(1, dtype=torch.int64, device=dev)
        self.status = torch.zeros(KB_STATUS_WORDS, dtype=torch.int32, device=dev)

    def run(self, conn, coords, coef, stage_events=None, stream=None):
        s = stream if stream is not None else torch.cuda.current_stream()
        ev = None
        if stage_events is not None:
            arr = (ctypes.c_void_p * len(stage_events))(*[int(e) for e in stage_events])
            self._ev_keep = arr
            ev = ctypes.cast(arr, ctypes.c_void_p)
        tu = self.tuning.to_c(ev)
        m = _mesh(self.elem, self.n_elem, self.n_node, conn, coords, coef, self.op)
        rc = _lib.lib().kb_build_lower_csr_grouped(ctypes.byref(m), self.prec, ctypes.byref(tu), self.group,
                                                   _ptr(self.ws), self.ws_bytes, _ptr(self.row_ptr),
                                                   _ptr(self.col_idx), _ptr(self.vals), self.cap, _ptr(self.nnz_dev),
                                                   _ptr(self.status), ctypes.c_void_p(s.cuda_stream))
        _check(rc, "kb_build_lower_csr_grouped")

    result = Builder.result


class StreamedGroupedBuilder:
    """Grouped build (Eq. 10) of a mesh whose connectivity and coefficients stay in host
    memory: only the group being built is on the device (the paper's upload of each
    group's data, Section 3).  Each group is copied from pinned host memory on a copy
    stream into one of two device staging buffers while the pass of the group before it
    runs on the compute stream (``kb_build_lower_csr_group_pass``); the node coordinates
    are device-resident.  The result equals ``GroupedBuilder``'s bit for bit.  ``run``
    allocates nothing."""

    def __init__(self, elem: int, n_elem: int, n_node: int, group_elems: int, cap: int, prec="fp32fb64",
                 tuning: Tuning | None = None, device="cuda", op="stiffness"):
        self.base = GroupedBuilder(elem, n_elem, n_node, group_elems, cap, prec, tuning, device, op)
        b = self.base
        self.n_groups = max(1, -(-b.n_elem // b.group)) if b.n_elem else 1
        gmax = min(b.group, max(b.n_elem, 1))
        dev = torch.device(device)
        self.stage_conn = [torch.empty((gmax, b.elem), dtype=torch.int32, device=dev) for _ in range(2)]
        self.stage_coef = [torch.empty(gmax, dtype=torch.float64, device=dev) for _ in range(2)]
        self.copy_stream = torch.cuda.Stream(device=dev)  # default priority
        self._free = [torch.cuda.Event(), torch.cuda.Event()]
        self._up = [torch.cuda.Event(), torch.cuda.Event()]

    def run(self, conn_host, coords, coef_host, stream=None):
        """Enqueue every pass; ``conn_host`` [n_elem, nen] int32 and ``coef_host`` [n_elem]
        float64 in pinned host memory, ``coords`` on the device."""
        b = self.base
        if conn_host.is_cuda or coef_host.is_cuda or not coords.is_cuda:
            raise ValueError("conn and coef must be host tensors, coords a device tensor")
        if not (conn_host.is_pinned() and coef_host.is_pinned()):
            raise ValueError("conn and coef must be in pinned host memory (torch pin_memory)")
        if conn_host.dtype != torch.int32 or conn_host.shape != (b.n_elem, b.elem) or not conn_host.is_contiguous():
            raise ValueError(f"conn must be a contiguous int32 [{b.n_elem}, {b.elem}] tensor")
        if coef_host.dtype != torch.float64 or coef_host.shape != (b.n_elem,) or not coef_host.is_contiguous():
            raise ValueError(f"coef must be a contiguous float64 [{b.n_elem}] tensor")
        if coords.dtype != torch.float64 or coords.shape != (b.n_node, 3) or not coords.is_contiguous():
            raise ValueError(f"coords must be a contiguous float64 [{b.n_node}, 3] tensor")
        compute = stream if stream is not None else torch.cuda.current_stream()
        L = _lib.lib()
        tu = b.tuning.to_c()
        m = _mesh(b.elem, b.n_elem, b.n_node, None, coords, None, b.op)
        for e in self._free:
            e.record(compute)
        for g in range(self.n_groups):
            k = g % 2
            e0 = g * b.group
            e1 = min(b.n_elem, e0 + b.group)
            with torch.cuda.stream(self.copy_stream):
                self.copy_stream.wait_event(self._free[k])  # the pass two groups back is done with it
                if e1 > e0:
                    self.stage_conn[k][: e1 - e0].copy_(conn_host[e0:e1], non_blocking=True)
                    self.stage_coef[k][: e1 - e0].copy_(coef_host[e0:e1], non_blocking=True)
                self._up[k].record(self.copy_stream)
            compute.wait_event(self._up[k])
            rc = L.kb_build_lower_csr_group_pass(ctypes.byref(m), b.prec, ctypes.byref(tu), b.group, g,
                                                 _ptr(self.stage_conn[k]), _ptr(self.stage_coef[k]), _ptr(b.ws),
                                                 b.ws_bytes, _ptr(b.row_ptr), _ptr(b.col_idx), _ptr(b.vals), b.cap,
                                                 _ptr(b.nnz_dev), _ptr(b.status), ctypes.c_void_p(compute.cuda_stream))
            _check(rc, "kb_build_lower_csr_group_pass")
            self._free[k].record(compute)

    def result(self, check: bool = True, allow_flags: int = 0) -> LowerCSR:
        return self.base.result(check=check, allow_flags=allow_flags)


def build_lower_csr_grouped(conn, coords, coef, elem: int, group_elems: int, cap: int, prec="fp32fb64",
                            tuning: Tuning | None = None, check=True, allow_flags: int = 0,
                            op="stiffness") -> LowerCSR:
    """Grouped construction (Eq. 10): elements in groups of ``group_elems``, the running
    sums carried from group to group; ``cap`` must be at least the final nnz."""
    _validate_mesh(conn, coords, coef, elem)
    b = GroupedBuilder(elem, conn.shape[0], coords.shape[0], group_elems, cap, prec, tuning, device=conn.device,
                       op=op)
    b.run(conn, coords, coef)
    return b.result(check=check, allow_flags=allow_flags)


def integrate_lower(conn, coords, coef, elem: int, prec="fp64", tuning: Tuning | None = None, check=True,
                    allow_flags: int = 0, op="stiffness"):
    """Per-element packed lower triangles [n_elem, nen(nen+1)/2] (Alg. 2 only)."""
    _validate_mesh(conn, coords, coef, elem)
    te = elem * (elem + 1) // 2
    out = torch.empty((conn.shape[0], te), dtype=value_dtype(prec), device=conn.device)
    status = torch.zeros(KB_STATUS_WORDS, dtype=torch.int32, device=conn.device)
    m = _mesh(elem, conn.shape[0], coords.shape[0], conn, coords, coef, op)
    tu = (tuning or Tuning()).to_c()
    rc = _lib.lib().kb_integrate_lower(ctypes.byref(m), _prec(prec), ctypes.byref(tu), _ptr(out), _ptr(status),
                                       ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    _check(rc, "kb_integrate_lower")
    torch.cuda.current_stream().synchronize()
    flags = int(status[0].item()) & 0xFFFFFFFF
    if check:
        _raise_on_flags(flags, allow_flags)
    return out, status


# ---- adjoint ---------------------------------------------------------------------------
class AdjointBuilder:
    """Reusable adjoint context for one mesh shape: workspace, gradients and status are
    allocated once, and ``run`` only enqueues kernels on the current stream."""

    def __init__(self, elem: int, n_elem: int, n_node: int, device="cuda"):
        self.elem, self.n_elem, self.n_node = int(elem), int(n_elem), int(n_node)
        m = _mesh(self.elem, self.n_elem, self.n_node)
        ws_bytes = ctypes.c_size_t(0)
        _check(_lib.lib().kb_plan_adjoint(ctypes.byref(m), ctypes.byref(ws_bytes)), "kb_plan_adjoint")
        self.ws_bytes = int(ws_bytes.value)
        dev = torch.device(device)
        self.ws = torch.empty(max(self.ws_bytes, 1), dtype=torch.uint8, device=dev)
        self.grad_coef = torch.empty(self.n_elem, dtype=torch.float64, device=dev)
        self.grad_coords = torch.empty((self.n_node, 3), dtype=torch.float64, device=dev)
        self.status = torch.zeros(KB_STATUS_WORDS, dtype=torch.int32, device=dev)

    def run(self, conn, coords, coef, row_ptr, col_idx, w):
        """Enqueue dL/dc and dL/dX of L = sum w_ij K_ij (w float64, one per pattern entry)."""
        _validate_mesh(conn, coords, coef, self.elem)
        if conn.shape[0] != self.n_elem or coords.shape[0] != self.n_node:
            raise ValueError("mesh shape differs from the one this context was made for")
        for name, t in (("row_ptr", row_ptr), ("col_idx", col_idx)):
            if t.dtype != torch.int32 or t.dim() != 1 or not t.is_contiguous() or t.device != conn.device:
                raise ValueError(f"{name} must be a contiguous int32 vector on the mesh's device")
        if row_ptr.numel() != self.n_node + 1:
            raise ValueError(f"row_ptr must have n_node + 1 = {self.n_node + 1} entries")
        if (w.dtype != torch.float64 or w.dim() != 1 or w.numel() != col_idx.numel() or not w.is_contiguous()
                or w.device != conn.device):
            raise ValueError("w must be a contiguous float64 device vector with one weight per pattern entry")
        m = _mesh(self.elem, self.n_elem, self.n_node, conn, coords, coef)
        rc = _lib.lib().kb_adjoint_lower(ctypes.byref(m), _ptr(row_ptr), _ptr(col_idx), _ptr(w), int(col_idx.numel()),
                                         _ptr(self.ws), self.ws_bytes, _ptr(self.grad_coef), _ptr(self.grad_coords),
                                         _ptr(self.status), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        _check(rc, "kb_adjoint_lower")

    def result(self, check: bool = True, allow_flags: int = 0):
        """Synchronise and return (dL/dc, dL/dX); raise on data errors if ``check``."""
        torch.cuda.current_stream().synchronize()
        if check:
            _raise_on_flags(int(self.status[0].item()) & 0xFFFFFFFF, allow_flags)
        return self.grad_coef, self.grad_coords


def adjoint_lower(conn, coords, coef, elem: int, row_ptr, col_idx, w, check=True, allow_flags: int = 0):
    """(dL/dc [n_elem], dL/dX [n_node, 3]) of L = sum w_ij K_ij over the lower pattern
    (row_ptr, col_idx) of this mesh's K, w (float64) aligned with that pattern.  FP64."""
    _validate_mesh(conn, coords, coef, elem)
    a = AdjointBuilder(elem, conn.shape[0], coords.shape[0], device=conn.device)
    a.run(conn, coords, coef, row_ptr, col_idx, w)
    if not check:
        return a.grad_coef, a.grad_coords
    return a.result(check=True, allow_flags=allow_flags)


class _LowerK(torch.autograd.Function):
    """Values of lower-triangular CSR K as a differentiable function of (coords, coef)."""

    @staticmethod
    def forward(ctx, coords, coef, conn, elem):
        r = build_lower_csr(conn, coords, coef, elem, prec="fp64")
        row_ptr, col_idx = r.row_ptr.clone(), r.col_idx.clone()
        ctx.save_for_backward(coords, coef, conn, row_ptr, col_idx)
        ctx.elem = elem
        ctx.mark_non_differentiable(row_ptr, col_idx)
        return r.vals.clone(), row_ptr, col_idx

    @staticmethod
    def backward(ctx, g_vals, _g_row_ptr, _g_col_idx):
        coords, coef, conn, row_ptr, col_idx = ctx.saved_tensors
        if g_vals is None:
            return None, None, None, None
        gc, gx = adjoint_lower(conn, coords, coef, ctx.elem, row_ptr, col_idx, g_vals.contiguous().to(torch.float64))
        return (gx if ctx.needs_input_grad[0] else None), (gc if ctx.needs_input_grad[1] else None), None, None


def lower_csr_values(coords, coef, conn, elem: int):
    """(vals, row_ptr, col_idx) of lower CSR K in FP64; vals is differentiable in coords and
    coef through the adjoint kernel (backward of any loss that is a function of vals)."""
    return _LowerK.apply(coords, coef, conn, elem)


# ---- batches -------------------------------------------------------------------------
@dataclass
class Batch:
    """Meshes packed back to back (device tensors): connectivity in mesh-local ids."""

    elem: int
    conn: torch.Tensor      # int32 [n_elem, nen]
    coords: torch.Tensor    # float64 [n_node, 3]
    coef: torch.Tensor      # float64 [n_elem]
    elem_off: torch.Tensor  # int64 [n_mesh + 1]
    node_off: torch.Tensor  # int64 [n_mesh + 1]
    elem_off_host: tuple = ()
    node_off_host: tuple = ()

    @property
    def n_mesh(self) -> int:
        return int(self.elem_off.numel()) - 1

    def to_c(self) -> KbBatch:
        return KbBatch(int(self.elem), self.n_mesh, int(self.conn.shape[0]), int(self.coords.shape[0]),
                       self.elem_off.data_ptr(), self.node_off.data_ptr(), self.conn.data_ptr(),
                       self.coords.data_ptr(), self.coef.data_ptr())


def pack_batch(meshes, elem: int, device="cuda") -> Batch:
    """Pack [(conn, coords, coef), ...] (array-likes, mesh-local ids) into one Batch."""
    import numpy as np

    conns, xs, cs, eo, no = [], [], [], [0], [0]
    for conn, coords, coef in meshes:
        conns.append(np.asarray(conn, dtype=np.int32).reshape(-1, elem))
        xs.append(np.asarray(coords, dtype=np.float64).reshape(-1, 3))
        cs.append(np.asarray(coef, dtype=np.float64).reshape(-1))
        eo.append(eo[-1] + conns[-1].shape[0])
        no.append(no[-1] + xs[-1].shape[0])
    dev = torch.device(device)
    cat = (lambda a, shape, dt: torch.from_numpy(np.concatenate(a) if a else np.zeros(shape, dtype=dt)).to(dev))
    return Batch(elem, cat(conns, (0, elem), np.int32), cat(xs, (0, 3), np.float64), cat(cs, (0,), np.float64),
                 torch.tensor(eo, dtype=torch.int64, device=dev), torch.tensor(no, dtype=torch.int64, device=dev),
                 tuple(eo), tuple(no))


def plan_batched(elem: int, n_mesh: int, n_elem: int, n_node: int, prec="fp32fb64", tuning: Tuning | None = None):
    ws = ctypes.c_size_t(0)
    nt = ctypes.c_int64(0)
    b = KbBatch(int(elem), int(n_mesh), int(n_elem), int(n_node), None, None, None, None, None)
    tu = (tuning or Tuning()).to_c()
    _check(_lib.lib().kb_plan_batched(ctypes.byref(b), _prec(prec), ctypes.byref(tu), ctypes.byref(ws),
                                      ctypes.byref(nt)), "kb_plan_batched")
    return int(ws.value), int(nt.value)


class BatchBuilder:
    """Reusable batched build: workspace and outputs allocated once for a batch shape.

    ``run`` enqueues the whole batch on the current stream and allocates nothing, so it
    can be captured in a HIP graph (``torch.cuda.graph``) and replayed.

    ``tuning="auto"`` takes the cached tuning for this batch's class of shapes, searched
    (and cached) first if there is none (``tune_batch``).
    """

    def __init__(self, batch: Batch, prec="fp32fb64", tuning: Tuning | str | None = None, cap: int | None = None,
                 tune_cache: str | None = None):
        self.batch = batch
        self.prec = _prec(prec)
        self.tune_entry = None
        if isinstance(tuning, str):
            if tuning != "auto":
                raise ValueError(f"tuning must be a Tuning, None or 'auto', not {tuning!r}")
            tuning, self.tune_entry = tune_batch(batch, prec, cache_path=tune_cache)
        self.tuning = tuning or Tuning()
        n_elem, n_node = int(batch.conn.shape[0]), int(batch.coords.shape[0])
        self.ws_bytes, self.n_triplets = plan_batched(batch.elem, batch.n_mesh, n_elem, n_node, self.prec, self.tuning)
        self.cap = self.n_triplets if cap is None else int(cap)
        dev = batch.conn.device
        self.ws = torch.empty(max(self.ws_bytes, 1), dtype=torch.uint8, device=dev)
        self.row_ptr = torch.empty(n_node + batch.n_mesh, dtype=torch.int32, device=dev)
        self.col_idx = torch.empty(max(self.cap, 1), dtype=torch.int32, device=dev)
        self.vals = torch.empty(max(self.cap, 1), dtype=value_dtype(self.prec), device=dev)
        self.nnz_off = torch.zeros(batch.n_mesh + 1, dtype=torch.int64, device=dev)
        self.status = torch.zeros(KB_STATUS_WORDS, dtype=torch.int32, device=dev)
        self._c = batch.to_c()

    def run(self, stream=None, stage_events=None):
        s = stream if stream is not None else torch.cuda.current_stream()
        ev = None
        if stage_events is not None:
            arr = (ctypes.c_void_p * len(stage_events))(*[int(e) for e in stage_events])
            self._ev_keep = arr
            ev = ctypes.cast(arr, ctypes.c_void_p)
        tu = self.tuning.to_c(ev)
        rc = _lib.lib().kb_build_lower_csr_batched(ctypes.byref(self._c), self.prec, ctypes.byref(tu), _ptr(self.ws),
                                                   self.ws_bytes, _ptr(self.row_ptr), _ptr(self.col_idx),
                                                   _ptr(self.vals), self.cap, _ptr(self.nnz_off), _ptr(self.status),
                                                   ctypes.c_void_p(s.cuda_stream))
        _check(rc, "kb_build_lower_csr_batched")

    def results(self, check: bool = True, allow_flags: int = 0) -> list:
        """Synchronise; one LowerCSR (views into the batch outputs) per mesh."""
        torch.cuda.current_stream().synchronize()
        flags = int(self.status[0].item()) & 0xFFFFFFFF
        if check:
            _raise_on_flags(flags, allow_flags)
        off = self.nnz_off.cpu().tolist()
        no = self.batch.node_off_host or tuple(self.batch.node_off.cpu().tolist())
        st = self.status.clone()
        out = []
        for m in range(self.batch.n_mesh):
            rp = self.row_ptr[no[m] + m: no[m + 1] + m + 1]
            ok = off[-1] <= self.cap
            out.append(LowerCSR(rp, self.col_idx[off[m]:off[m + 1]] if ok else self.col_idx[:0],
                                self.vals[off[m]:off[m + 1]] if ok else self.vals[:0], off[m + 1] - off[m], st))
        return out


def tune_batch(batch: Batch, prec="fp32fb64", cache_path: str | None = None, refresh: bool = False):
    """(Tuning, cache entry) for this batch: the cached choice for its (architecture,
    element, precision, size class), else a timed search over the tile, bucket, sub-bucket
    and segment knobs, stored in the JSON cache (``autotune``)."""
    from . import autotune

    n_pairs = int(batch.conn.shape[0]) * batch.elem * (batch.elem + 1) // 2

    def make_run(t):
        b = BatchBuilder(batch, prec, t)
        return b.run

    return autotune.tuned("batch", batch.elem, prec, n_pairs, make_run, cache_path=cache_path, refresh=refresh)


def tune_build(conn, coords, coef, elem: int, prec="fp32fb64", op="stiffness", cache_path: str | None = None,
               refresh: bool = False):
    """(Tuning, cache entry) for builds of one mesh of this shape: the cached choice for
    its (architecture, operator, element, precision, size class), else a timed search
    over the tile, bucket, sub-bucket, segment and table knobs on this mesh, stored in
    the JSON cache (``autotune``).  Every candidate gives the same matrix bit for bit."""
    from . import autotune

    n_elem, n_node = int(conn.shape[0]), int(coords.shape[0])
    n_pairs = n_elem * elem * (elem + 1) // 2

    def make_run(t):
        b = Builder(elem, n_elem, n_node, prec, t, device=conn.device, op=op)
        return lambda: b.run(conn, coords, coef)

    kind = "build" if _op(op) == KB_OP_STIFFNESS else "build-mass"
    return autotune.tuned(kind, elem, prec, n_pairs, make_run, cache_path=cache_path, refresh=refresh)


def build_lower_csr_batched(meshes, elem: int, prec="fp32fb64", tuning: Tuning | None = None, check=True,
                            allow_flags: int = 0, device="cuda") -> list:
    """Build each mesh of [(conn, coords, coef), ...] (mesh-local ids) in one batched call."""
    b = BatchBuilder(pack_batch(meshes, elem, device), prec, tuning)
    b.run()
    return b.results(check=check, allow_flags=allow_flags)


__all__ = ["Builder", "BatchBuilder", "Batch", "GroupedBuilder", "StreamedGroupedBuilder", "LowerCSR", "KBuildError", "Tuning", "build_lower_csr",
           "build_lower_csr_noalloc", "lower_csr_tensor",
           "build_lower_csr_batched", "assemble_lower_csr", "integrate_lower", "adjoint_lower", "AdjointBuilder",
           "lower_csr_values",
           "pack_batch", "plan", "plan_batched",
           "tune_batch", "tune_build", "status_string", "version", "value_dtype", "STAGE_NAMES", "KB_N_STAGES",
           "KB_HEX8", "KB_TET4", "KB_FP64", "KB_FP32", "KB_FP32_FB64", "KB_OP_STIFFNESS", "KB_OP_MASS"]
