"""FP64 CPU oracle for the lower-triangular Poisson stiffness matrix (test infrastructure).

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this package; the product path never does.  It wraps the plain C oracle
in ``kb_oracle.c`` (built by ``oracle/build.py``) and shares nothing with the
HIP library.  ``oracle.dense`` holds a second, independent dense route for tiny
meshes.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

F_INDEX, F_REPEAT, F_INVERTED, F_NONFINITE = 1, 2, 4, 8

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        i64, i32, p = ctypes.c_int64, ctypes.c_int, ctypes.c_void_p
        L.orc_gauss_rule.argtypes = [i32, p, p]
        L.orc_gauss_rule.restype = i32
        L.orc_element_lower.argtypes = [i32, i32, p, ctypes.c_double, p]
        L.orc_element_lower.restype = i32
        L.orc_integrate_lower.argtypes = [i32, i64, i64, p, p, p, p]
        L.orc_integrate_lower.restype = i64
        L.orc_assemble_lower_csr.argtypes = [i32, i64, i64, p, p, p, p, p, i64, p]
        L.orc_assemble_lower_csr.restype = i64
        L.orc_build_lower_csr.argtypes = [i32, i64, i64, p, p, p, p, p, p, i64, p]
        L.orc_build_lower_csr.restype = i64
        L.orc_rows_lower.argtypes = [i32, i64, i64, p, p, p, i64, p, p, p, p, i64]
        L.orc_rows_lower.restype = i64
        L.orc_element_mass_lower.argtypes = [i32, p, ctypes.c_double, p]
        L.orc_element_mass_lower.restype = i32
        L.orc_integrate_mass_lower.argtypes = [i32, i64, i64, p, p, p, p]
        L.orc_integrate_mass_lower.restype = i64
        L.orc_assemble_lower_csr_dof.argtypes = [i32, i32, i64, i64, p, p, p, p, p, i64, p]
        L.orc_assemble_lower_csr_dof.restype = i64
        L.orc_adjoint_lower.argtypes = [i32, i64, i64, p, p, p, p, p, p, p, p]
        L.orc_adjoint_lower.restype = i64
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def gauss_rule(n: int):
    x = np.zeros(5)
    w = np.zeros(5)
    if lib().orc_gauss_rule(n, _p(x), _p(w)) != 0:
        raise ValueError(n)
    return x[:n].copy(), w[:n].copy()


def element_lower(elem: int, X, c: float = 1.0, gauss_n: int = 2):
    """Lower triangle (packed, p = a(a+1)/2 + b) of one element matrix and its flags."""
    X = _c(X, np.float64).reshape(elem, 3)
    out = np.zeros(elem * (elem + 1) // 2)
    r = lib().orc_element_lower(elem, gauss_n, _p(X), float(c), _p(out))
    if r < 0:
        raise ValueError("bad element arguments")
    return out, int(r)


def unpack_lower(klow: np.ndarray, nen: int) -> np.ndarray:
    """Full symmetric nen x nen matrix from packed lower storage."""
    K = np.zeros(klow.shape[:-1] + (nen, nen))
    for a in range(nen):
        for b in range(a + 1):
            K[..., a, b] = klow[..., a * (a + 1) // 2 + b]
            K[..., b, a] = klow[..., a * (a + 1) // 2 + b]
    return K


def integrate_lower(elem, conn, coords, coef):
    conn = _c(conn, np.int32)
    coords = _c(coords, np.float64)
    coef = _c(coef, np.float64)
    nel = conn.shape[0]
    T = elem * (elem + 1) // 2
    out = np.zeros((nel, T))
    r = lib().orc_integrate_lower(elem, nel, coords.shape[0], _p(conn), _p(coords), _p(coef), _p(out))
    if r < 0:
        raise ValueError("bad arguments")
    return out, int(r)


def _csr_call(fn, n_row, cap, *args):
    row_ptr = np.zeros(n_row + 1, np.int32)
    col = np.zeros(max(cap, 1), np.int32)
    val = np.zeros(max(cap, 1))
    flags = np.zeros(1, np.uint32)
    nnz = fn(*args, _p(row_ptr), _p(col), _p(val), cap, _p(flags))
    if nnz < 0:
        raise ValueError("bad arguments")
    if nnz > cap:
        raise RuntimeError("capacity")
    return row_ptr, col[:nnz], val[:nnz], int(flags[0])


def build_lower_csr(elem, conn, coords, coef):
    """Alg. 1 in FP64: returns (row_ptr, col_idx, vals, flags)."""
    conn = _c(conn, np.int32)
    coords = _c(coords, np.float64)
    coef = _c(coef, np.float64)
    nn = coords.shape[0]
    cap = conn.shape[0] * elem * (elem + 1) // 2
    return _csr_call(lib().orc_build_lower_csr, nn, cap, elem, conn.shape[0], nn, _p(conn), _p(coords), _p(coef))


def assemble_lower_csr(elem, conn, n_node, klow):
    conn = _c(conn, np.int32)
    klow = _c(klow, np.float64)
    cap = conn.shape[0] * elem * (elem + 1) // 2
    return _csr_call(lib().orc_assemble_lower_csr, n_node, cap, elem, conn.shape[0], n_node, _p(conn), _p(klow))


def rows_lower(elem, conn, coords, coef, rows):
    """Entries of the selected rows (CSR in the given row order)."""
    conn = _c(conn, np.int32)
    coords = _c(coords, np.float64)
    coef = _c(coef, np.float64)
    rows = _c(rows, np.int32)
    n_sel = rows.shape[0]
    cap = 64 * elem * max(n_sel, 1) * 4
    ptr = np.zeros(n_sel + 1, np.int32)
    col = np.zeros(cap, np.int32)
    val = np.zeros(cap)
    n = lib().orc_rows_lower(elem, conn.shape[0], coords.shape[0], _p(conn), _p(coords), _p(coef), n_sel,
                             _p(rows), _p(ptr), _p(col), _p(val), cap)
    if n < 0:
        raise ValueError("bad arguments")
    if n > cap:
        raise RuntimeError("capacity")
    return ptr, col[:n], val[:n]


def build_mesh(mesh):
    return build_lower_csr(mesh.elem, mesh.conn, mesh.coords, mesh.coef)


_par = None


def par_build_mesh(mesh, threads: int = 0):
    """The oracle's construction on ``threads`` host threads (0: all), for timing: the
    same element routine, parallel loops and sort (``timing_par.c``).  Returns
    (row_ptr, col_idx, vals, flags); values agree with build_mesh to rounding."""
    global _par
    if _par is None:
        if not os.path.exists(_build.PAR_LIB):
            _build.build()
        L = ctypes.CDLL(_build.PAR_LIB)
        i64, i32, p = ctypes.c_int64, ctypes.c_int, ctypes.c_void_p
        L.orc_par_build_lower_csr.argtypes = [i32, i64, i64, p, p, p, p, p, p, i64, p, i32]
        L.orc_par_build_lower_csr.restype = i64
        L.orc_par_max_threads.argtypes = []
        L.orc_par_max_threads.restype = i32
        _par = L
    conn = _c(mesh.conn, np.int32)
    coords = _c(mesh.coords, np.float64)
    coef = _c(mesh.coef, np.float64)
    nn = coords.shape[0]
    cap = conn.shape[0] * mesh.elem * (mesh.elem + 1) // 2
    row_ptr = np.zeros(nn + 1, np.int32)
    col = np.zeros(max(cap, 1), np.int32)
    val = np.zeros(max(cap, 1))
    flags = np.zeros(1, np.uint32)
    nnz = _par.orc_par_build_lower_csr(mesh.elem, conn.shape[0], nn, _p(conn), _p(coords), _p(coef), _p(row_ptr),
                                       _p(col), _p(val), cap, _p(flags), int(threads))
    if nnz < 0:
        raise ValueError("bad arguments")
    return row_ptr, col[:nnz], val[:nnz], int(flags[0])


def par_threads() -> int:
    """Threads the all-cores harness uses by default (OpenMP's count on this host)."""
    if _par is None:
        par_build_mesh(type("M", (), dict(elem=4, conn=np.zeros((0, 4), np.int32), coords=np.zeros((0, 3)),
                                          coef=np.zeros(0)))())
    return int(_par.orc_par_max_threads())


def adjoint_lower(mesh, row_ptr, col_idx, w):
    """(dL/dc [n_elem], dL/dX [n_node, 3]) of L = sum W_ij K_ij over the lower pattern
    (row_ptr, col_idx) of the mesh's K, W aligned with that pattern.  FP64."""
    conn = _c(mesh.conn, np.int32)
    gc = np.zeros(mesh.n_elem)
    gx = np.zeros((mesh.n_node, 3))
    r = lib().orc_adjoint_lower(mesh.elem, mesh.n_elem, mesh.n_node, _p(conn), _p(_c(mesh.coords, np.float64)),
                                _p(_c(mesh.coef, np.float64)), _p(_c(row_ptr, np.int32)), _p(_c(col_idx, np.int32)),
                                _p(_c(w, np.float64)), _p(gc), _p(gx))
    if r < 0:
        raise ValueError("element pair outside the given pattern")
    return gc, gx, int(r)


def element_mass_lower(elem: int, X, rho: float = 1.0):
    """Packed lower triangle of one element's consistent mass matrix and its flags."""
    X = _c(X, np.float64)
    out = np.zeros(elem * (elem + 1) // 2)
    f = lib().orc_element_mass_lower(elem, _p(X), float(rho), _p(out))
    if f < 0:
        raise ValueError("bad element")
    return out, int(f)


def integrate_mass_lower(elem, conn, coords, coef):
    conn = _c(conn, np.int32)
    T = elem * (elem + 1) // 2
    out = np.zeros((conn.shape[0], T))
    f = lib().orc_integrate_mass_lower(elem, conn.shape[0], coords.shape[0], _p(conn), _p(_c(coords, np.float64)),
                                       _p(_c(coef, np.float64)), _p(out))
    if f < 0:
        raise ValueError("bad element type")
    return out, int(f)


def build_mass_mesh(mesh):
    """Lower CSR of the consistent mass matrix: element values, then the oracle assembly."""
    mlow, f = integrate_mass_lower(mesh.elem, mesh.conn, mesh.coords, mesh.coef)
    rp, col, val, f2 = assemble_lower_csr(mesh.elem, mesh.conn, mesh.n_node, mlow)
    return rp, col, val, f | f2


def assemble_lower_csr_dof(elem, dof, conn, n_node, klow):
    """Lower CSR (dof * n_node rows) of element matrices with dof components per node."""
    conn = _c(conn, np.int32)
    klow = _c(klow, np.float64)
    nd = elem * dof
    cap = conn.shape[0] * nd * (nd + 1) // 2
    return _csr_call(lib().orc_assemble_lower_csr_dof, dof * n_node, cap, elem, dof, conn.shape[0], n_node, _p(conn),
                     _p(klow))
