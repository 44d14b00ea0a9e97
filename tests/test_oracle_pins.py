"""Pins of the FP64 oracle to facts fixed by the paper and by the mathematics.

Every check here is independent of the oracle's own code: closed-form element
matrices, the paper's printed Table 1 / Table 2 numbers, invariants of the weak
form (zero row sums, positive semidefiniteness, the energy of linear fields),
a second dense route written with different mathematics (``oracle.dense``), and
brute-force properties on tiny meshes.  Each is chosen so that a plausible
mistake in the oracle (a dropped term, a wrong sign or index, a transposed
Jacobian, a lost duplicate) fails at least one of them.
"""
from __future__ import annotations

import numpy as np
import pytest

import meshgen
import oracle
from oracle import dense
from tests.helpers import (csr_diag, full_row_sums, load_table, lower_to_dense, scaled_error, sym_quad)

RNG = np.random.default_rng(12345)


# ----------------------------------------------------------------- quadrature
@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_gauss_rule_exact_degree(n):
    """An n-point Gauss-Legendre rule is exact for degree <= 2n-1 and not for 2n."""
    x, w = oracle.gauss_rule(n)
    for k in range(2 * n + 1):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        got = float(np.sum(w * x ** k))
        if k <= 2 * n - 1:
            assert abs(got - exact) < 1e-14
        else:
            assert abs(got - exact) > 1e-6


def test_gauss_rule_two_point_is_paper_rule():
    x, w = oracle.gauss_rule(2)
    np.testing.assert_allclose(x, [-1 / np.sqrt(3), 1 / np.sqrt(3)], rtol=0, atol=1e-16)
    np.testing.assert_allclose(w, [1.0, 1.0], rtol=0, atol=0)


# ------------------------------------------------------- closed-form elements
HEX_IJK = meshgen.HEX_CORNERS


def hex_box_closed_form(hx, hy, hz, c):
    """Trilinear brick on an axis-aligned hx*hy*hz box, exact integrals.

    k_ab = c V sum_d (s_d / h_d^2) prod_{d' != d} m_d', with s_d = +1 if a and b
    share their coordinate along d, else -1, and m = 1/3 if shared, else 1/6.
    """
    h = np.array([hx, hy, hz])
    V = hx * hy * hz
    K = np.zeros((8, 8))
    for a in range(8):
        for b in range(8):
            same = HEX_IJK[a] == HEX_IJK[b]
            m = np.where(same, 1 / 3, 1 / 6)
            s = np.where(same, 1.0, -1.0)
            K[a, b] = c * V * sum(s[d] / h[d] ** 2 * np.prod(np.delete(m, d)) for d in range(3))
    return K


def box_corners(hx, hy, hz, origin=(0, 0, 0)):
    return HEX_IJK * np.array([hx, hy, hz]) + np.array(origin)


def test_hex_unit_cube_values():
    """Cube of edge h: diagonal c h/3, edge 0, face and body diagonals -c h/12."""
    h, c = 0.37, 2.5
    K = oracle.unpack_lower(oracle.element_lower(8, box_corners(h, h, h), c)[0], 8)
    for a in range(8):
        for b in range(8):
            nd = int(np.sum(HEX_IJK[a] != HEX_IJK[b]))
            want = {0: c * h / 3, 1: 0.0, 2: -c * h / 12, 3: -c * h / 12}[nd]
            assert abs(K[a, b] - want) < 1e-15 * c


@pytest.mark.parametrize("trial", range(5))
def test_hex_box_closed_form(trial):
    hx, hy, hz = RNG.uniform(0.05, 3.0, 3)
    c = float(np.exp(RNG.uniform(-5, 5)))
    org = RNG.uniform(-10, 10, 3)
    klow, flags = oracle.element_lower(8, box_corners(hx, hy, hz, org), c)
    assert flags == 0
    want = hex_box_closed_form(hx, hy, hz, c)
    got = oracle.unpack_lower(klow, 8)
    scale = np.sqrt(np.outer(np.diag(want), np.diag(want)))
    assert np.max(np.abs(got - want) / scale) < 1e-13


def test_tet_reference_element():
    """Reference tet: (c/6) [[3,-1,-1,-1],[-1,1,0,0],[-1,0,1,0],[-1,0,0,1]]."""
    X = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], float)
    c = 3.0
    got = oracle.unpack_lower(oracle.element_lower(4, X, c)[0], 4)
    want = c / 6 * np.array([[3, -1, -1, -1], [-1, 1, 0, 0], [-1, 0, 1, 0], [-1, 0, 0, 1]])
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-15)


def _random_hex(jitter=0.25):
    X = box_corners(1, 1, 1) + RNG.uniform(-jitter, jitter, (8, 3))
    A = np.linalg.qr(RNG.standard_normal((3, 3)))[0] * RNG.uniform(0.3, 3)
    if np.linalg.det(A) < 0:
        A[:, 0] *= -1
    return X @ A.T + RNG.uniform(-5, 5, 3)


def _random_tet():
    while True:
        X = RNG.standard_normal((4, 3))
        if np.linalg.det(np.hstack([np.ones((4, 1)), X])) > 0.05:
            return X


@pytest.mark.parametrize("trial", range(8))
def test_distorted_elements_match_dense_route(trial):
    """Distorted (non-affine, sheared, rotated) elements: cofactor route == numpy.linalg route."""
    for elem, X in ((8, _random_hex()), (4, _random_tet())):
        c = float(np.exp(RNG.uniform(-3, 3)))
        klow, flags = oracle.element_lower(elem, X, c)
        assert flags == 0
        got = oracle.unpack_lower(klow, elem)
        want = dense.element_full(elem, X, c)
        scale = np.sqrt(np.outer(np.diag(want), np.diag(want)))
        assert np.max(np.abs(got - want) / scale) < 1e-12


def test_affine_hex_two_point_rule_is_exact():
    """Parallelepiped bricks: the 2x2x2 rule equals a 5x5x5 rule; distorted ones differ."""
    A = RNG.standard_normal((3, 3)) + 3 * np.eye(3)
    X = box_corners(1, 1, 1) @ A.T
    k2 = oracle.element_lower(8, X, 1.0, gauss_n=2)[0]
    k5 = oracle.element_lower(8, X, 1.0, gauss_n=5)[0]
    assert np.max(np.abs(k2 - k5)) < 1e-13 * np.max(np.abs(k5))
    Xd = _random_hex(0.3)
    d2 = oracle.element_lower(8, Xd, 1.0, gauss_n=2)[0]
    d5 = oracle.element_lower(8, Xd, 1.0, gauss_n=5)[0]
    assert np.max(np.abs(d2 - d5)) > 1e-8 * np.max(np.abs(d5))


@pytest.mark.parametrize("elem", [8, 4])
def test_element_invariances(elem):
    """Linearity in c, rigid-motion invariance, k(sX) = s k(X), zero row sums, PSD."""
    X = _random_hex() if elem == 8 else _random_tet()
    k1 = oracle.unpack_lower(oracle.element_lower(elem, X, 1.0)[0], elem)
    k7 = oracle.unpack_lower(oracle.element_lower(elem, X, 7.0)[0], elem)
    np.testing.assert_allclose(k7, 7.0 * k1, rtol=1e-14, atol=1e-14 * np.abs(k1).max())
    Q = np.linalg.qr(RNG.standard_normal((3, 3)))[0]
    if np.linalg.det(Q) < 0:
        Q[:, 0] *= -1
    kr = oracle.unpack_lower(oracle.element_lower(elem, X @ Q.T + 4.0, 1.0)[0], elem)
    np.testing.assert_allclose(kr, k1, rtol=0, atol=1e-12 * np.abs(k1).max())
    ks = oracle.unpack_lower(oracle.element_lower(elem, 2.5 * X, 1.0)[0], elem)
    np.testing.assert_allclose(ks, 2.5 * k1, rtol=0, atol=1e-13 * np.abs(k1).max())
    assert np.max(np.abs(k1.sum(axis=1))) < 1e-13 * np.abs(k1).max()
    assert np.linalg.eigvalsh(k1).min() > -1e-13 * np.abs(k1).max()


# ----------------------------------------------------------- printed numbers
def hex_nnz(n):
    """nnz of lower-triangular K of an N^3 brick grid, n = N + 1 nodes per axis."""
    return ((3 * n - 2) ** 3 + n ** 3) // 2


def test_table1_closed_form_and_byte_model():
    """Every NNZ and MB figure of Table 1 follows from the grid; oracle reproduces the small ones."""
    t = load_table("table1.txt")
    for nel, ntrip, nnz, comp, mb_t, mb_c, save in t:
        N = round(nel ** (1 / 3))
        assert N ** 3 == nel
        n = N + 1
        assert 36 * nel == ntrip
        assert hex_nnz(n) == nnz
        assert round(100 * (1 - nnz / ntrip), 1) == pytest.approx(comp)
        # triplet: int32 row + int32 col + double value = 16 B; CSC: 16 B per nnz + 8 B per column pointer
        mb_trip = 16 * ntrip / 1e6
        mb_csc = (16 * nnz + 8 * (n ** 3 + 1)) / 1e6
        digits = 2 if mb_t < 10 else 1
        assert round(mb_trip, digits) == pytest.approx(mb_t)
        assert round(mb_csc, 2 if mb_c < 10 else 1) == pytest.approx(mb_c)
        assert round(100 * (1 - mb_csc / mb_trip), 1) == pytest.approx(save)


@pytest.mark.parametrize("N", [10, 20])
def test_oracle_reproduces_table1_nnz(N):
    t = load_table("table1.txt")
    want = int(t[t[:, 0] == N ** 3][0, 2])
    m = meshgen.box_mesh(8, N)
    rp, col, val, flags = oracle.build_mesh(m)
    assert flags == 0
    assert rp[-1] == want == len(col)


def test_table2_matrix_sizes():
    for nel, nn in load_table("table2.txt"):
        N = round(nel ** (1 / 3))
        assert meshgen.counts(8, N)[:2] == (int(nel), int(nn))


@pytest.mark.parametrize("N", [1, 2, 3, 5])
def test_kuhn_tet_nnz(N):
    """Kuhn-split grid: nnz of lower K = (2n-1)^3, and T = 10 nel."""
    m = meshgen.box_mesh(4, N, jitter=0.1, seed=7)
    rp, col, val, flags = oracle.build_mesh(m)
    assert flags == 0
    assert len(col) == (2 * (N + 1) - 1) ** 3


# -------------------------------------------------------- global invariants
def _mesh(elem, N, **kw):
    base = dict(jitter=0.25, coef=(1e-2, 1e2), permute_nodes=True, permute_elems=True, seed=11)
    base.update(kw)
    return meshgen.box_mesh(elem, N, **base)


@pytest.mark.parametrize("elem", [8, 4])
def test_lower_structure(elem):
    """Rows ascend, columns ascend within a row, diagonal last, all col <= row."""
    m = _mesh(elem, 4)
    rp, col, val, _ = oracle.build_mesh(m)
    for i in range(m.n_node):
        c = col[rp[i]:rp[i + 1]]
        assert np.all(np.diff(c) > 0)
        assert len(c) > 0 and c[-1] == i


@pytest.mark.parametrize("elem", [8, 4])
def test_zero_row_sums(elem):
    """Constants lie in the null space of K: every full row sums to zero."""
    m = _mesh(elem, 6)
    rp, col, val, _ = oracle.build_mesh(m)
    d = csr_diag(rp, col, val, m.n_node)
    s = full_row_sums(rp, col, val, m.n_node)
    assert np.max(np.abs(s) / d) < 1e-12


@pytest.mark.parametrize("elem", [8, 4])
def test_psd_dense(elem):
    m = _mesh(elem, 3)
    rp, col, val, _ = oracle.build_mesh(m)
    K = lower_to_dense(rp, col, val, m.n_node)
    ev = np.linalg.eigvalsh(K)
    assert ev.min() > -1e-12 * ev.max()
    # exactly one zero mode (connected mesh, no boundary conditions)
    assert np.sum(ev < 1e-9 * ev.max()) == 1


@pytest.mark.parametrize("elem", [8, 4])
def test_energy_of_linear_fields_unit_cube(elem):
    """u = g.x + u0 on the unit cube with c = 1: u^T K u = |g|^2 (boundary nodes fixed)."""
    m = meshgen.box_mesh(elem, 6, jitter=0.3, coef=1.0, permute_nodes=True, permute_elems=True, seed=3)
    rp, col, val, _ = oracle.build_mesh(m)
    for _ in range(3):
        g = RNG.standard_normal(3)
        u = m.coords @ g + RNG.standard_normal()
        assert sym_quad(rp, col, val, u) == pytest.approx(float(g @ g), rel=1e-12)


def _element_volume_independent(elem, X):
    if elem == 4:
        return np.linalg.det(np.hstack([np.ones((4, 1)), X])) / 6.0
    # divergence theorem over the six bilinear faces: V = 1/3 sum_faces int x . (x_u x x_v) du dv,
    # integrated with a 4x4 rule (the integrand is polynomial of degree <= 3 per variable)
    faces = [(0, 3, 2, 1), (4, 5, 6, 7), (0, 1, 5, 4), (1, 2, 6, 5), (2, 3, 7, 6), (3, 0, 4, 7)]
    g, w = np.polynomial.legendre.leggauss(4)
    V = 0.0
    for f in faces:
        P = X[list(f)]
        for ui, u in enumerate(g):
            for vi, v in enumerate(g):
                s, t = (u + 1) / 2, (v + 1) / 2
                x = (1 - s) * (1 - t) * P[0] + s * (1 - t) * P[1] + s * t * P[2] + (1 - s) * t * P[3]
                xu = ((1 - t) * (P[1] - P[0]) + t * (P[2] - P[3])) / 2
                xv = ((1 - s) * (P[3] - P[0]) + s * (P[2] - P[1])) / 2
                V += w[ui] * w[vi] * x @ np.cross(xu, xv) / 3
    return V


@pytest.mark.parametrize("elem", [8, 4])
def test_energy_of_linear_fields_variable_c(elem):
    """u^T K u = |g|^2 sum_e c_e V_e with V_e computed independently of the oracle."""
    m = _mesh(elem, 3, jitter=0.3)
    rp, col, val, _ = oracle.build_mesh(m)
    vol = np.array([_element_volume_independent(elem, m.coords[E]) for E in m.conn])
    g = RNG.standard_normal(3)
    u = m.coords @ g - 0.7
    want = float(g @ g) * float(np.sum(m.coef * vol))
    assert sym_quad(rp, col, val, u) == pytest.approx(want, rel=1e-12)


@pytest.mark.parametrize("elem,N", [(8, 2), (8, 3), (4, 2), (4, 3)])
def test_dense_brute_force(elem, N):
    """Sparse triplet route == dense full-matrix route (pattern exact, values 1e-13 scaled)."""
    m = _mesh(elem, N)
    rp, col, val, flags = oracle.build_mesh(m)
    assert flags == 0
    K = dense.dense_K(elem, m.conn, m.coords, m.coef)
    P = dense.dense_pattern(elem, m.conn, m.n_node)
    drp, dcol, dval = dense.to_lower_csr(K, P)
    np.testing.assert_array_equal(rp, drp)
    np.testing.assert_array_equal(col, dcol)
    assert scaled_error(rp, col, val, dval) < 1e-13


@pytest.mark.parametrize("elem", [8, 4])
def test_permutation_equivariance(elem):
    """Relabelling nodes relabels and re-lowers K; reordering elements leaves K unchanged."""
    m = _mesh(elem, 4, permute_nodes=False, permute_elems=False)
    rp, col, val, _ = oracle.build_mesh(m)
    K = lower_to_dense(rp, col, val, m.n_node)
    perm = RNG.permutation(m.n_node)
    conn2 = perm[m.conn]
    coords2 = np.empty_like(m.coords)
    coords2[perm] = m.coords
    ep = RNG.permutation(m.n_elem)
    rp2, col2, val2, _ = oracle.build_lower_csr(elem, conn2[ep], coords2, m.coef[ep])
    K2 = lower_to_dense(rp2, col2, val2, m.n_node)
    np.testing.assert_allclose(K2[np.ix_(perm, perm)], K, rtol=0, atol=1e-13 * np.abs(K).max())
    # element order alone: identical pattern
    rp3, col3, val3, _ = oracle.build_lower_csr(elem, m.conn[ep], m.coords, m.coef[ep])
    np.testing.assert_array_equal(rp3, rp)
    np.testing.assert_array_equal(col3, col)
    assert scaled_error(rp, col, val3, val) < 1e-14


def test_assembly_from_element_values_matches_full_build():
    m = _mesh(4, 4)
    klow, _ = oracle.integrate_lower(m.elem, m.conn, m.coords, m.coef)
    a = oracle.assemble_lower_csr(m.elem, m.conn, m.n_node, klow)
    b = oracle.build_mesh(m)
    for x, y in zip(a[:3], b[:3]):
        np.testing.assert_array_equal(x, y)


def test_rows_lower_matches_full_build():
    m = _mesh(8, 5)
    rp, col, val, _ = oracle.build_mesh(m)
    rows = RNG.choice(m.n_node, 17, replace=False).astype(np.int32)
    sp, sc, sv = oracle.rows_lower(m.elem, m.conn, m.coords, m.coef, rows)
    for k, r in enumerate(rows):
        np.testing.assert_array_equal(sc[sp[k]:sp[k + 1]], col[rp[r]:rp[r + 1]])
        np.testing.assert_allclose(sv[sp[k]:sp[k + 1]], val[rp[r]:rp[r + 1]], rtol=1e-14, atol=0)


# ----------------------------------------------------------------- data flags
def test_flags():
    m = _mesh(4, 2)
    conn = m.conn.copy()
    conn[3, 2] = m.n_node  # out of range
    assert oracle.build_lower_csr(4, conn, m.coords, m.coef)[3] & oracle.F_INDEX
    conn = m.conn.copy()
    conn[5, 1] = conn[5, 0]  # repeated node
    assert oracle.build_lower_csr(4, conn, m.coords, m.coef)[3] & oracle.F_REPEAT
    conn = m.conn.copy()
    conn[7, [2, 3]] = conn[7, [3, 2]]  # inverted tet
    assert oracle.build_lower_csr(4, conn, m.coords, m.coef)[3] == oracle.F_INVERTED
    coords = m.coords.copy()
    coords[m.conn[0, 0], 1] = np.nan
    assert oracle.build_lower_csr(4, m.conn, coords, m.coef)[3] & oracle.F_NONFINITE
    coef = m.coef.copy()
    coef[2] = np.inf
    assert oracle.build_lower_csr(4, m.conn, m.coords, coef)[3] & oracle.F_NONFINITE
