"""Second, independent oracle route for tiny meshes (test infrastructure only).

Dense FP64 assembly of the FULL element matrices into an ``n_node x n_node``
array (Eq. 6, K = sum_e k_e), after which the lower triangle is taken.  It shares
no arithmetic with ``kb_oracle.c``: no triplets, no sort, no packed lower
storage, and different mathematics for each step:

* hex8: shape functions as tensor products of the 1D linear Lagrange pair
  (1 -+ x)/2, the Gauss-Legendre rule from ``numpy.polynomial.legendre.leggauss``,
  the Jacobian with ``einsum``, its inverse and determinant from ``numpy.linalg``
  (Eq. 8-9 of Section 2);
* tet4: barycentric gradients from the inverse of the 4x4 matrix
  [[1, x, y, z], ...] and the volume from its determinant, k = c V G^T G
  (the gradient of a linear function is constant, so no quadrature is needed).
"""
from __future__ import annotations

import numpy as np

# local corner -> (i, j, k) in {0,1}^3: same corner order as the mesh generator
_HEX_IJK = np.array([(0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0), (0, 0, 1), (1, 0, 1), (1, 1, 1), (0, 1, 1)])


def _lagrange1(x):
    """Values and derivatives of the 1D pair l0 = (1-x)/2, l1 = (1+x)/2."""
    v = np.stack([(1 - x) / 2, (1 + x) / 2], axis=-1)
    d = np.stack([-0.5 * np.ones_like(x), 0.5 * np.ones_like(x)], axis=-1)
    return v, d


def hex_full(X: np.ndarray, c: float = 1.0, n: int = 2) -> np.ndarray:
    """Full 8x8 brick matrix with an n^3 Gauss rule (X is 8 x 3)."""
    g, w = np.polynomial.legendre.leggauss(n)
    K = np.zeros((8, 8))
    for a_, r in enumerate(g):
        for b_, s in enumerate(g):
            for c_, t in enumerate(g):
                vr, dr = _lagrange1(np.array(r))
                vs, ds = _lagrange1(np.array(s))
                vt, dt = _lagrange1(np.array(t))
                i, j, k = _HEX_IJK[:, 0], _HEX_IJK[:, 1], _HEX_IJK[:, 2]
                dN = np.stack([dr[i] * vs[j] * vt[k], vr[i] * ds[j] * vt[k], vr[i] * vs[j] * dt[k]])  # 3 x 8
                J = np.einsum("ia,aj->ij", dN, X)
                G = np.linalg.inv(J) @ dN  # physical gradients, 3 x 8
                K += w[a_] * w[b_] * w[c_] * np.linalg.det(J) * (G.T @ G)
    return c * K


def tet_full(X: np.ndarray, c: float = 1.0) -> np.ndarray:
    """Full 4x4 linear tet matrix (X is 4 x 3)."""
    M = np.hstack([np.ones((4, 1)), X])  # rows [1, x, y, z]
    V = np.linalg.det(M) / 6.0
    G = np.linalg.inv(M)[1:, :]  # 3 x 4: gradients of the barycentric coordinates
    return c * V * (G.T @ G)


def element_full(elem: int, X: np.ndarray, c: float = 1.0) -> np.ndarray:
    return hex_full(X, c) if elem == 8 else tet_full(X, c)


def dense_K(elem: int, conn: np.ndarray, coords: np.ndarray, coef: np.ndarray) -> np.ndarray:
    """Full symmetric global matrix (n_node x n_node) by dense summation."""
    nn = coords.shape[0]
    K = np.zeros((nn, nn))
    for e in range(conn.shape[0]):
        E = conn[e]
        ke = element_full(elem, coords[E], coef[e])
        K[np.ix_(E, E)] += ke
    return K


def dense_pattern(elem: int, conn: np.ndarray, n_node: int) -> np.ndarray:
    """Boolean structural pattern of the full K (independent of values)."""
    P = np.zeros((n_node, n_node), dtype=bool)
    for E in conn:
        P[np.ix_(E, E)] = True
    return P


def to_lower_csr(K: np.ndarray, P: np.ndarray):
    """Lower-triangular CSR (structural pattern P, zeros kept) of a dense matrix."""
    L = np.tril(P)
    rows, cols = np.nonzero(L)  # row-major order: rows ascend, columns ascend within a row
    row_ptr = np.zeros(K.shape[0] + 1, np.int64)
    np.add.at(row_ptr, rows + 1, 1)
    return np.cumsum(row_ptr).astype(np.int32), cols.astype(np.int32), K[rows, cols]


# ---- consistent mass matrix (second route) ---------------------------------------------
def hex_mass_full(X: np.ndarray, rho: float = 1.0, n: int = 2) -> np.ndarray:
    """Full 8x8 brick mass matrix rho * int N N^T dV with an n^3 Gauss rule."""
    g, w = np.polynomial.legendre.leggauss(n)
    M = np.zeros((8, 8))
    i, j, k = _HEX_IJK[:, 0], _HEX_IJK[:, 1], _HEX_IJK[:, 2]
    for a_, r in enumerate(g):
        for b_, s in enumerate(g):
            for c_, t in enumerate(g):
                vr, dr = _lagrange1(np.array(r))
                vs, ds = _lagrange1(np.array(s))
                vt, dt = _lagrange1(np.array(t))
                N = vr[i] * vs[j] * vt[k]
                dN = np.stack([dr[i] * vs[j] * vt[k], vr[i] * ds[j] * vt[k], vr[i] * vs[j] * dt[k]])
                J = np.einsum("ia,aj->ij", dN, X)
                M += w[a_] * w[b_] * w[c_] * np.linalg.det(J) * np.outer(N, N)
    return rho * M


def tet_mass_full(X: np.ndarray, rho: float = 1.0, n: int = 4) -> np.ndarray:
    """Full 4x4 tet mass matrix by a collapsed-coordinate (Duffy) Gauss rule on the
    reference tet, r = u, s = v (1 - u), t = w (1 - u)(1 - v), Jacobian (1 - u)^2 (1 - v),
    scaled by the affine map's determinant."""
    g, wt = np.polynomial.legendre.leggauss(n)
    x, wx = (g + 1) / 2, wt / 2  # on [0, 1]
    M = np.zeros((4, 4))
    for iu, u in enumerate(x):
        for iv, v in enumerate(x):
            for iw, w_ in enumerate(x):
                r, s, t = u, v * (1 - u), w_ * (1 - u) * (1 - v)
                N = np.array([1 - r - s - t, r, s, t])
                M += wx[iu] * wx[iv] * wx[iw] * (1 - u) ** 2 * (1 - v) * np.outer(N, N)
    D = np.linalg.det((X[1:] - X[0]).T)
    return rho * D * M


def dense_M(elem: int, conn: np.ndarray, coords: np.ndarray, coef: np.ndarray) -> np.ndarray:
    nn = coords.shape[0]
    M = np.zeros((nn, nn))
    for e in range(conn.shape[0]):
        E = conn[e]
        me = hex_mass_full(coords[E], coef[e]) if elem == 8 else tet_mass_full(coords[E], coef[e])
        M[np.ix_(E, E)] += me
    return M
