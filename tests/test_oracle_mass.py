"""Pins of the oracle's consistent mass matrix (another integrand through the same
construction: the closing remark of Section 5).  Closed forms, total mass against an
independent divergence-theorem volume, a second numpy route (tensor Gauss for the brick,
a collapsed-coordinate rule for the tet), invariances, definiteness, and planted mistakes.
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
from tests.test_oracle_pins import _element_volume_independent

RNG = np.random.default_rng(17)
BOX = np.array([(0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0), (0, 0, 1), (1, 0, 1), (1, 1, 1), (0, 1, 1)], float)
REF_TET = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], float)


def distorted(elem, seed):
    r = np.random.default_rng(seed)
    X = (BOX if elem == 8 else REF_TET) + 0.15 * r.uniform(-1, 1, (elem, 3))
    return X


def test_box_closed_form():
    """Axis-aligned brick h1 x h2 x h3: m_ab = rho V / 216 * prod_d (1 + [a_d = b_d])."""
    h = np.array([0.5, 1.3, 2.0])
    X = BOX * h
    rho = 3.0
    M = oracle.unpack_lower(oracle.element_mass_lower(8, X, rho)[0], 8)
    V = float(np.prod(h))
    for a in range(8):
        for b in range(8):
            want = rho * V / 216 * np.prod([2 if BOX[a, d] == BOX[b, d] else 1 for d in range(3)])
            assert M[a, b] == pytest.approx(want, rel=1e-14)


def test_reference_tet_closed_form():
    M = oracle.unpack_lower(oracle.element_mass_lower(4, REF_TET, 1.0)[0], 4)
    np.testing.assert_allclose(M, (np.ones((4, 4)) + np.eye(4)) / 120.0, rtol=1e-15)


@pytest.mark.parametrize("elem", [8, 4])
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_total_mass_is_rho_times_volume(elem, seed):
    """sum_ab M_ab = rho V (the shape functions sum to 1), V from the divergence theorem."""
    X = distorted(elem, seed)
    rho = 1.7
    M = oracle.unpack_lower(oracle.element_mass_lower(elem, X, rho)[0], elem)
    assert M.sum() == pytest.approx(rho * _element_volume_independent(elem, X), rel=1e-13)


@pytest.mark.parametrize("elem", [8, 4])
@pytest.mark.parametrize("seed", [4, 5])
def test_second_route(elem, seed):
    X = distorted(elem, seed)
    M = oracle.unpack_lower(oracle.element_mass_lower(elem, X, 0.9)[0], elem)
    D = dense.hex_mass_full(X, 0.9) if elem == 8 else dense.tet_mass_full(X, 0.9)
    np.testing.assert_allclose(M, D, rtol=1e-13, atol=1e-15 * np.abs(D).max())


def test_affine_brick_rule_is_exact():
    """On an affine (parallelepiped) brick the 2x2x2 rule equals a 4x4x4 rule."""
    A = np.array([[1.0, 0.2, 0.1], [0.0, 0.9, 0.3], [0.1, -0.2, 1.2]])
    X = BOX @ A.T + 0.3
    M = oracle.unpack_lower(oracle.element_mass_lower(8, X, 1.0)[0], 8)
    np.testing.assert_allclose(M, dense.hex_mass_full(X, 1.0, n=4), rtol=1e-13)


@pytest.mark.parametrize("elem", [8, 4])
def test_invariances_and_scaling(elem):
    X = distorted(elem, 6)
    M = oracle.unpack_lower(oracle.element_mass_lower(elem, X, 1.0)[0], elem)
    q, _ = np.linalg.qr(RNG.standard_normal((3, 3)))
    q *= np.sign(np.linalg.det(q))
    Mr = oracle.unpack_lower(oracle.element_mass_lower(elem, X @ q.T + 5.0, 1.0)[0], elem)
    np.testing.assert_allclose(Mr, M, rtol=1e-12)
    Ms = oracle.unpack_lower(oracle.element_mass_lower(elem, 2.5 * X, 4.0)[0], elem)
    np.testing.assert_allclose(Ms, 4.0 * 2.5 ** 3 * M, rtol=1e-12)


@pytest.mark.parametrize("elem", [8, 4])
def test_assembled_mass_positive_definite_and_total(elem):
    m = meshgen.box_mesh(elem, 3, 2, 2, jitter=0.25, coef=(0.5, 2.0), permute_nodes=True, permute_elems=True,
                         seed=8)
    rp, col, val, f = oracle.build_mass_mesh(m)
    assert f == 0
    n = m.n_node
    Mfull = np.zeros((n, n))
    rows = np.repeat(np.arange(n), np.diff(rp))
    Mfull[rows, col] = val
    Mfull = Mfull + np.tril(Mfull, -1).T
    assert np.linalg.eigvalsh(Mfull).min() > 0
    vol = np.array([_element_volume_independent(elem, m.coords[E]) for E in m.conn])
    assert Mfull.sum() == pytest.approx(float(np.sum(m.coef * vol)), rel=1e-12)
    np.testing.assert_allclose(Mfull, dense.dense_M(elem, m.conn, m.coords, m.coef), rtol=1e-12,
                               atol=1e-14 * np.abs(Mfull).max())


MUTANTS = {
    "tet_offdiagonal_factor": ("V * (a == b ? 2.0 : 1.0) / 20.0", "V * (a == b ? 2.0 : 1.0) / 24.0"),
    "tet_volume_factor": ("double V = det / 6.0;", "double V = det;"),
    "brick_shape_product": ("mlow[a * (a + 1) / 2 + b] += W * det * N[a] * N[b];",
                            "mlow[a * (a + 1) / 2 + b] += W * det * N[a];"),
    "brick_determinant_dropped": ("mlow[a * (a + 1) / 2 + b] += W * det * N[a] * N[b];",
                                  "mlow[a * (a + 1) / 2 + b] += W * N[a] * N[b];"),
    "brick_shape_sign": ("N[a] = (1.0 + HEX_NAT[a][0] * r) * (1.0 + HEX_NAT[a][1] * s)",
                         "N[a] = (1.0 - HEX_NAT[a][0] * r) * (1.0 + HEX_NAT[a][1] * s)"),
    "density_dropped": ("mlow[p] *= rho;", "mlow[p] *= 1.0;"),
}


def _lib(tmp_path, name, src):
    c = tmp_path / f"{name}.c"
    c.write_text(src)
    so = tmp_path / f"lib{name}.so"
    subprocess.run(["gcc", "-std=c11", "-O1", "-fPIC", "-shared", "-o", str(so), str(c), "-lm"], check=True)
    L = ctypes.CDLL(str(so))
    L.orc_element_mass_lower.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p]
    L.orc_element_mass_lower.restype = ctypes.c_int
    return L


def _passes(L):
    for elem in (8, 4):
        for seed in (1, 2):
            X = np.ascontiguousarray(distorted(elem, seed))
            out = np.zeros(elem * (elem + 1) // 2)
            L.orc_element_mass_lower(elem, X.ctypes.data_as(ctypes.c_void_p), 1.3, out.ctypes.data_as(ctypes.c_void_p))
            M = oracle.unpack_lower(out, elem)
            D = dense.hex_mass_full(X, 1.3) if elem == 8 else dense.tet_mass_full(X, 1.3)
            if not np.allclose(M, D, rtol=1e-12, atol=1e-14):
                return False
            if abs(M.sum() - 1.3 * _element_volume_independent(elem, X)) > 1e-12:
                return False
    return True


def test_unmodified_mass_source_passes(tmp_path):
    assert _passes(_lib(tmp_path, "orig", open(SRC).read()))


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mass_mutant_is_caught(tmp_path, name):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, name
    assert not _passes(_lib(tmp_path, name, src.replace(old, new))), name
