"""Pins of the oracle's assembly with several degrees of freedom per node (Alg. 1's
Mapping with DOFxn > 1): one DOF equals the scalar assembly; element matrices k ⊗ I_d
assemble to K ⊗ I_d; a dense numpy assembly of full element matrices agrees; node
relabelling permutes rows and columns consistently.
"""
from __future__ import annotations

import numpy as np
import pytest

import meshgen
import oracle


def small(elem, seed):
    return meshgen.box_mesh(elem, 3, 2, 2, jitter=0.2, coef=(0.5, 2.0), permute_nodes=True, permute_elems=True,
                            seed=seed)


def random_klow(n_elem, nd, seed):
    """Random symmetric element matrices, packed lower (p(p+1)/2 + q)."""
    return meshgen.element_matrices(n_elem, nd, seed)


def unpack(k, nd):
    M = np.zeros((nd, nd))
    for p in range(nd):
        for q in range(p + 1):
            M[p, q] = M[q, p] = k[p * (p + 1) // 2 + q]
    return M


def dense_lower(elem, dof, conn, n_node, klow):
    nd = elem * dof
    n = dof * n_node
    K = np.zeros((n, n))
    P = np.zeros((n, n), bool)
    for e, E in enumerate(conn):
        g = np.array([dof * E[p // dof] + p % dof for p in range(nd)])
        K[np.ix_(g, g)] += unpack(klow[e], nd)
        P[np.ix_(g, g)] = True
    L = np.tril(P)
    rows, cols = np.nonzero(L)
    rp = np.zeros(n + 1, np.int64)
    np.add.at(rp, rows + 1, 1)
    return np.cumsum(rp), cols, K[rows, cols]


@pytest.mark.parametrize("elem", [8, 4])
def test_one_dof_is_the_scalar_assembly(elem):
    m = small(elem, 1)
    klow, _ = oracle.integrate_lower(m.elem, m.conn, m.coords, m.coef)
    a = oracle.assemble_lower_csr_dof(elem, 1, m.conn, m.n_node, klow)
    b = oracle.assemble_lower_csr(elem, m.conn, m.n_node, klow)
    for x, y in zip(a[:3], b[:3]):
        np.testing.assert_array_equal(x, y)


@pytest.mark.parametrize("elem", [8, 4])
@pytest.mark.parametrize("dof", [2, 3])
def test_kronecker_identity(elem, dof):
    """k_e ⊗ I_d per element gives K ⊗ I_d: row dof*i + c holds K_ij at column dof*j + c."""
    m = small(elem, 2)
    k1, _ = oracle.integrate_lower(m.elem, m.conn, m.coords, m.coef)
    nd = elem * dof
    kd = np.zeros((m.n_elem, nd * (nd + 1) // 2))
    for e in range(m.n_elem):
        full = np.kron(oracle.unpack_lower(k1[e], elem), np.eye(dof))
        kd[e] = [full[p, q] for p in range(nd) for q in range(p + 1)]
    rp, col, val, f = oracle.assemble_lower_csr_dof(elem, dof, m.conn, m.n_node, kd)
    srp, scol, sval, _ = oracle.build_mesh(m)
    n = dof * m.n_node
    got = np.zeros((n, n))
    got[np.repeat(np.arange(n), np.diff(rp)), col] = val
    want = np.zeros((n, n))
    S = np.zeros((m.n_node, m.n_node))
    S[np.repeat(np.arange(m.n_node), np.diff(srp)), scol] = sval
    for c in range(dof):
        want[c::dof, c::dof] = S
    np.testing.assert_allclose(np.tril(got), np.tril(want), rtol=1e-13, atol=1e-15 * np.abs(want).max())


@pytest.mark.parametrize("elem", [8, 4])
@pytest.mark.parametrize("dof", [2, 3])
def test_dense_assembly(elem, dof):
    m = small(elem, 3)
    klow = random_klow(m.n_elem, elem * dof, 4)
    rp, col, val, f = oracle.assemble_lower_csr_dof(elem, dof, m.conn, m.n_node, klow)
    drp, dcol, dval = dense_lower(elem, dof, m.conn, m.n_node, klow)
    np.testing.assert_array_equal(rp, drp)
    np.testing.assert_array_equal(col, dcol)
    np.testing.assert_allclose(val, dval, rtol=1e-13, atol=1e-13)


def test_relabelling_permutes_consistently():
    elem, dof = 4, 3
    m = small(elem, 5)
    klow = random_klow(m.n_elem, elem * dof, 6)
    rp, col, val, _ = oracle.assemble_lower_csr_dof(elem, dof, m.conn, m.n_node, klow)
    perm = np.random.default_rng(7).permutation(m.n_node)
    rp2, col2, val2, _ = oracle.assemble_lower_csr_dof(elem, dof, perm[m.conn], m.n_node, klow)
    n = dof * m.n_node
    A = np.zeros((n, n))
    A[np.repeat(np.arange(n), np.diff(rp)), col] = val
    A = A + np.tril(A, -1).T
    B = np.zeros((n, n))
    B[np.repeat(np.arange(n), np.diff(rp2)), col2] = val2
    B = B + np.tril(B, -1).T
    g = (dof * perm[:, None] + np.arange(dof)[None, :]).reshape(-1)  # old DOF -> new DOF
    np.testing.assert_allclose(B[np.ix_(g, g)], A, rtol=1e-13, atol=1e-13)
