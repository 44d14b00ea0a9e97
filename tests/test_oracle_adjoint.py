"""Pins of the oracle's adjoint (dL/dc, dL/dX of L = sum W_ij K_ij over the lower
pattern).  The adjoint is not in the paper; it is derived from Eq. 7-9, so it is pinned
to what the mathematics fixes, with code independent of it:

* finite differences of L computed by the dense second route (numpy, full element
  matrices; no packed storage, no triplets) along random directions;
* linearity in c (dL/dc_e = L_e / c_e, so sum_e c_e dL/dc_e = L);
* invariances of K: translation (sum of node gradients 0), rotation (sum of x × g 0)
  and degree-1 homogeneity in the coordinates (sum of x · g = L);
* planted mistakes in a copy of the C source are caught by these checks.
"""
from __future__ import annotations

import ctypes
import subprocess

import numpy as np
import pytest

import meshgen
import oracle
from oracle import dense
from oracle.build import SRC


def small(elem, seed, n=3):
    return meshgen.box_mesh(elem, n, n - 1, n + 1, jitter=0.25, coef=(0.1, 10.0), permute_nodes=True,
                            permute_elems=True, seed=seed)


def dense_loss(elem, conn, coords, coef, rp, col, w):
    """L = sum W_ij K_ij with K from the dense second route."""
    K = dense.dense_K(elem, conn, coords, coef)
    rows = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
    return float(np.sum(w * K[rows, col]))


def setup(elem, seed):
    m = small(elem, seed)
    rp, col, val, fl = oracle.build_mesh(m)
    w = np.random.default_rng(seed).standard_normal(len(col))
    return m, rp, col, val, w


@pytest.mark.parametrize("elem", [8, 4])
def test_linear_in_coefficient(elem):
    m, rp, col, val, w = setup(elem, 1)
    gc, gx, f = oracle.adjoint_lower(m, rp, col, w)
    L = float(w @ val)
    assert f == 0
    assert abs(float(m.coef @ gc) - L) <= 1e-12 * max(1.0, abs(L))
    # one element's coefficient moved: the loss moves by exactly its derivative times the step
    e = 5
    c2 = m.coef.copy()
    c2[e] *= 1.5
    L2 = dense_loss(elem, m.conn, m.coords, c2, rp, col, w)
    assert abs((L2 - L) - 0.5 * m.coef[e] * gc[e]) <= 1e-10 * max(1.0, abs(L))


@pytest.mark.parametrize("elem", [8, 4])
def test_finite_differences_in_coordinates(elem):
    """Central differences (h = 1e-6 of the cell size) of the dense route's loss along
    random directions agree with the directional derivative to 1e-6 relative."""
    m, rp, col, val, w = setup(elem, 2)
    gc, gx, f = oracle.adjoint_lower(m, rp, col, w)
    rng = np.random.default_rng(3)
    h = 1e-6 * m.meta["h"]
    for _ in range(4):
        v = rng.standard_normal(m.coords.shape)
        Lp = dense_loss(elem, m.conn, m.coords + h * v, m.coef, rp, col, w)
        Lm = dense_loss(elem, m.conn, m.coords - h * v, m.coef, rp, col, w)
        fd = (Lp - Lm) / (2 * h)
        an = float(np.sum(gx * v))
        assert abs(fd - an) <= 1e-6 * max(abs(an), np.abs(gx).sum() * 1e-3)


@pytest.mark.parametrize("elem", [8, 4])
def test_single_node_single_component(elem):
    """Finite difference of one coordinate of one interior node."""
    m, rp, col, val, w = setup(elem, 4)
    gc, gx, f = oracle.adjoint_lower(m, rp, col, w)
    h = 1e-6 * m.meta["h"]
    node = int(np.argmax(np.abs(gx[:, 1])))
    Xp, Xm = m.coords.copy(), m.coords.copy()
    Xp[node, 1] += h
    Xm[node, 1] -= h
    fd = (dense_loss(elem, m.conn, Xp, m.coef, rp, col, w) - dense_loss(elem, m.conn, Xm, m.coef, rp, col, w)) / (2 * h)
    assert abs(fd - gx[node, 1]) <= 1e-6 * abs(gx[node, 1])


@pytest.mark.parametrize("elem", [8, 4])
def test_invariances(elem):
    m, rp, col, val, w = setup(elem, 5)
    gc, gx, f = oracle.adjoint_lower(m, rp, col, w)
    L = float(w @ val)
    scale = np.abs(gx).sum()
    # translation: K does not change when every node moves by the same vector
    assert np.abs(gx.sum(axis=0)).max() <= 1e-12 * scale
    # rotation: nor under a rigid rotation (isotropic coefficient)
    torque = np.cross(m.coords, gx).sum(axis=0)
    assert np.abs(torque).max() <= 1e-12 * scale * np.abs(m.coords).max()
    # scaling: K is homogeneous of degree 1 in the coordinates (|J| ~ s^3, B ~ 1/s)
    assert abs(float(np.sum(m.coords * gx)) - L) <= 1e-11 * max(1.0, abs(L), scale)


def test_zero_weights_give_zero_gradients():
    m, rp, col, val, w = setup(8, 6)
    gc, gx, f = oracle.adjoint_lower(m, rp, col, np.zeros_like(w))
    assert not gc.any() and not gx.any()


def test_pattern_mismatch_is_an_error():
    m, rp, col, val, w = setup(4, 7)
    col2 = col.copy()
    col2[-1] = col2[-1] - 1 if col2[-1] > 0 else 1  # the last row loses its diagonal
    with pytest.raises(ValueError):
        oracle.adjoint_lower(m, rp, col2, w)


# ---- planted mistakes ---------------------------------------------------------------
MUTANTS = {
    "off_diagonal_weight_not_halved": ("S[a][b] = a == b ? w[k] : 0.5 * w[k];", "S[a][b] = w[k];"),
    "trace_term_dropped": ("double s = tr * B[i][a];", "double s = 0.0;"),
    "factor_two_dropped": ("s -= 2.0 * B[j][a] * M[j][i];", "s -= B[j][a] * M[j][i];"),
    "coefficient_dropped": ("G[a][i] += c * W * det * s;", "G[a][i] += W * det * s;"),
    "determinant_dropped_in_dc": ("*gc += W * det * tr;", "*gc += W * tr;"),
    "gradient_to_wrong_node": ("grad_coords[(int64_t)E[a] * 3 + j] += G[a][j];",
                               "grad_coords[(int64_t)E[(a + 1) % nen] * 3 + j] += G[a][j];"),
    "inverse_not_transposed": ("for (int j = 0; j < 3; ++j) s += Ji[i][j] * dN[j][a];\n      B[i][a] = s;\n    }\n  /* M",
                               "for (int j = 0; j < 3; ++j) s += Ji[j][i] * dN[j][a];\n      B[i][a] = s;\n    }\n  /* M"),
}


def _mutant_lib(tmp_path, name, src):
    c = tmp_path / f"{name}.c"
    c.write_text(src)
    so = tmp_path / f"lib{name}.so"
    subprocess.run(["gcc", "-std=c11", "-O1", "-fPIC", "-shared", "-o", str(so), str(c), "-lm"], check=True)
    L = ctypes.CDLL(str(so))
    p, i32, i64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64
    L.orc_adjoint_lower.argtypes = [i32, i64, i64, p, p, p, p, p, p, p, p]
    L.orc_adjoint_lower.restype = i64
    return L


def _checks_pass(L, elem):
    """The compact set of independent checks, on one small permuted mesh."""
    m = small(elem, 11)
    rp, col, val, fl = oracle.build_mesh(m)
    w = np.random.default_rng(12).standard_normal(len(col))
    gc, gx = np.zeros(m.n_elem), np.zeros((m.n_node, 3))
    P = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
    conn = np.ascontiguousarray(m.conn, np.int32)
    r = L.orc_adjoint_lower(elem, m.n_elem, m.n_node, P(conn), P(m.coords), P(m.coef), P(rp), P(col), P(w), P(gc),
                            P(gx))
    if r < 0:
        return False
    L0 = float(w @ val)
    if abs(float(m.coef @ gc) - L0) > 1e-10 * max(1.0, abs(L0)):
        return False
    h = 1e-6 * m.meta["h"]
    v = np.random.default_rng(13).standard_normal(m.coords.shape)
    fd = (dense_loss(elem, m.conn, m.coords + h * v, m.coef, rp, col, w)
          - dense_loss(elem, m.conn, m.coords - h * v, m.coef, rp, col, w)) / (2 * h)
    an = float(np.sum(gx * v))
    return abs(fd - an) <= 1e-6 * max(abs(an), np.abs(gx).sum() * 1e-3)


def test_unmodified_source_passes(tmp_path):
    src = open(SRC).read()
    L = _mutant_lib(tmp_path, "orig", src)
    assert _checks_pass(L, 8) and _checks_pass(L, 4)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, name
    L = _mutant_lib(tmp_path, name, src.replace(old, new))
    assert not (_checks_pass(L, 8) and _checks_pass(L, 4)), name
