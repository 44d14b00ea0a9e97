"""The pins must catch plausible mistakes in the oracle.

Each case plants one mistake in a temporary copy of ``oracle/kb_oracle.c``
(CPU only), builds it with gcc and runs a compact set of the independent checks
(dense second route on distorted elements, closed-form brick, energy of linear
fields, dense brute force of a tiny permuted mesh).  At least one check must fail
for every mutant, and all must pass for the unmodified source.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np
import pytest

import meshgen
from oracle import dense
from oracle.build import SRC

MUTANTS = {
    "transposed_jacobian": ("J[i][j] = s;", "J[j][i] = s;"),
    "det_sign_term": ("- J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0])",
                      "+ J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0])"),
    "inverse_entry": ("Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;",
                      "Ji[1][2] = (J[0][0] * J[1][2] - J[0][2] * J[1][0]) / det;"),
    "inverse_not_transposed": ("s += Ji[i][j] * dN[j][a];", "s += Ji[j][i] * dN[j][a];"),
    "dropped_weight": ("klow[a * (a + 1) / 2 + b] += W * det * s;", "klow[a * (a + 1) / 2 + b] += det * s;"),
    "abs_free_det_dropped": ("klow[a * (a + 1) / 2 + b] += W * det * s;", "klow[a * (a + 1) / 2 + b] += W * s;"),
    "dropped_coef": ("klow[p] *= c;", "klow[p] *= 1.0;"),
    "shape_derivative_sign": ("dN[1][a] = (1.0 + ra * r) * sa * (1.0 + ta * t) / 8.0;",
                              "dN[1][a] = (1.0 - ra * r) * sa * (1.0 + ta * t) / 8.0;"),
    "wrong_gauss_point": ("x[0] = -1.0 / sqrt(3.0); x[1] = 1.0 / sqrt(3.0);",
                          "x[0] = -0.5; x[1] = 0.5;"),
    "packed_index": ("klow[a * (a + 1) / 2 + b] += W * det * s;", "klow[b * (b + 1) / 2 + a % (b + 1)] += W * det * s;"),
    "row_is_min": ("uint32_t row = i > j ? i : j, col = i > j ? j : i;",
                   "uint32_t row = i > j ? j : i, col = i > j ? i : j;"),
    "duplicate_not_summed": ("if (nnz <= cap) vals[k] += t[i].val;", "if (nnz <= cap) vals[k] = t[i].val;"),
    "tet_weight": ("double det = add_point(4, dN, X, 1.0 / 6.0, klow);", "double det = add_point(4, dN, X, 1.0, klow);"),
}


def _build(tmp_path, name, src):
    c = tmp_path / f"{name}.c"
    c.write_text(src)
    so = tmp_path / f"lib{name}.so"
    subprocess.run(["gcc", "-std=c11", "-O1", "-fPIC", "-shared", "-o", str(so), str(c), "-lm"], check=True)
    L = ctypes.CDLL(str(so))
    p, i32, i64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64
    L.orc_element_lower.argtypes = [i32, i32, p, ctypes.c_double, p]
    L.orc_element_lower.restype = i32
    L.orc_build_lower_csr.argtypes = [i32, i64, i64, p, p, p, p, p, p, i64, p]
    L.orc_build_lower_csr.restype = i64
    return L


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _elem(L, elem, X, c):
    X = np.ascontiguousarray(X, np.float64)
    out = np.zeros(elem * (elem + 1) // 2)
    L.orc_element_lower(elem, 2, _ptr(X), float(c), _ptr(out))
    K = np.zeros((elem, elem))
    for a in range(elem):
        for b in range(a + 1):
            K[a, b] = K[b, a] = out[a * (a + 1) // 2 + b]
    return K


def _build_csr(L, m):
    conn = np.ascontiguousarray(m.conn, np.int32)
    cap = m.n_elem * m.elem * (m.elem + 1) // 2
    rp = np.zeros(m.n_node + 1, np.int32)
    col = np.zeros(cap, np.int32)
    val = np.zeros(cap)
    fl = np.zeros(1, np.uint32)
    nnz = L.orc_build_lower_csr(m.elem, m.n_elem, m.n_node, _ptr(conn), _ptr(m.coords), _ptr(m.coef),
                                _ptr(rp), _ptr(col), _ptr(val), cap, _ptr(fl))
    return rp, col[:nnz], val[:nnz]


def _checks(L) -> list[str]:
    """Names of the independent checks that fail for library L."""
    failed = []
    rng = np.random.default_rng(5)
    # 1. distorted elements vs the numpy.linalg dense route
    Xh = meshgen.HEX_CORNERS + rng.uniform(-0.25, 0.25, (8, 3))
    Xh = Xh @ np.array([[1.0, 0.3, 0.1], [0.2, 1.1, -0.2], [0.1, 0.0, 0.9]]).T
    Xt = np.array([[0.1, 0.0, 0.2], [1.0, 0.2, 0.1], [0.3, 1.1, 0.0], [0.2, 0.1, 0.8]])
    for elem, X in ((8, Xh), (4, Xt)):
        got, want = _elem(L, elem, X, 1.7), dense.element_full(elem, X, 1.7)
        if not np.allclose(got, want, rtol=1e-10, atol=1e-10 * np.abs(want).max()):
            failed.append(f"dense_route_{elem}")
    # 2. axis-aligned closed form (cube of edge h: diag h/3, face/body diag -h/12, edge 0)
    h = 0.5
    K = _elem(L, 8, meshgen.HEX_CORNERS * h, 2.0)
    if abs(K[0, 0] - 2.0 * h / 3) > 1e-13 or abs(K[0, 6] + 2.0 * h / 12) > 1e-13:
        failed.append("closed_form")
    # 3. tiny permuted jittered mesh: sparse route vs dense route, and energy of a linear field
    for elem in (8, 4):
        m = meshgen.box_mesh(elem, 2, jitter=0.25, coef=(0.1, 10), permute_nodes=True, permute_elems=True, seed=2)
        rp, col, val = _build_csr(L, m)
        Kd = dense.dense_K(elem, m.conn, m.coords, m.coef)
        P = dense.dense_pattern(elem, m.conn, m.n_node)
        drp, dcol, dval = dense.to_lower_csr(Kd, P)
        if len(col) != len(dcol) or not np.array_equal(col, dcol) or not np.allclose(val, dval, rtol=1e-10, atol=1e-12):
            failed.append(f"dense_mesh_{elem}")
        m1 = meshgen.box_mesh(elem, 3, jitter=0.3, coef=1.0, seed=4)
        rp, col, val = _build_csr(L, m1)
        g = np.array([0.3, -1.2, 0.7])
        u = m1.coords @ g
        rows = np.repeat(np.arange(m1.n_node), np.diff(rp))
        q = np.sum(np.where(rows == col, 1.0, 2.0) * val * u[rows] * u[col])
        if abs(q - g @ g) > 1e-10:
            failed.append(f"energy_{elem}")
    return failed


def test_unmodified_oracle_passes_checks(tmp_path):
    src = open(SRC).read()
    assert _checks(_build(tmp_path, "orig", src)) == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation site for {name} not found"
    L = _build(tmp_path, name, src.replace(old, new, 1))
    assert _checks(L), f"mutant {name} was not caught by any pin"
