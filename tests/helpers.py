"""Shared test helpers (comparison metrics only; no element arithmetic)."""
from __future__ import annotations

import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load_table(name: str) -> np.ndarray:
    return np.loadtxt(os.path.join(GOLDEN, name), comments="#")


def csr_diag(row_ptr, col, val, n):
    """Diagonal of a lower CSR whose rows end with the diagonal entry (0 if absent)."""
    d = np.zeros(n)
    rp = np.asarray(row_ptr, np.int64)
    last = rp[1:n + 1] - 1
    has = (rp[1:n + 1] > rp[:n])
    idx = np.nonzero(has)[0]
    ok = idx[np.asarray(col)[last[idx]] == idx]
    d[ok] = np.asarray(val, np.float64)[last[ok]]
    return d


def csr_rows(row_ptr):
    rp = np.asarray(row_ptr, np.int64)
    return np.repeat(np.arange(len(rp) - 1), np.diff(rp))


def scaled_error(row_ptr, col, val_a, val_b, diag=None):
    """max |a_ij - b_ij| / sqrt(K_ii K_jj), with K_ii taken from b (the reference).

    Each element matrix is PSD, so |K_ij| <= sqrt(K_ii K_jj) and this scale is the
    natural one for entries that cancel to ~0.
    """
    n = len(row_ptr) - 1
    if diag is None:
        diag = csr_diag(row_ptr, col, val_b, n)
    rows = csr_rows(row_ptr)
    scale = np.sqrt(np.abs(diag[rows] * diag[col]))
    scale = np.where(scale > 0, scale, 1.0)
    if len(val_a) == 0:
        return 0.0
    return float(np.max(np.abs(np.asarray(val_a, np.float64) - np.asarray(val_b, np.float64)) / scale))


def lower_to_dense(row_ptr, col, val, n):
    K = np.zeros((n, n))
    rows = csr_rows(row_ptr)
    K[rows, col] = val
    return K + np.tril(K, -1).T


def full_row_sums(row_ptr, col, val, n):
    """Row sums of the full symmetric K from its lower CSR."""
    rows = csr_rows(row_ptr)
    s = np.zeros(n)
    np.add.at(s, rows, val)
    off = rows != col
    np.add.at(s, col[off], np.asarray(val)[off])
    return s


def sym_quad(row_ptr, col, val, u):
    """u^T K u from the lower CSR of symmetric K."""
    rows = csr_rows(row_ptr)
    v = np.asarray(val, np.float64)
    w = np.where(rows == col, 1.0, 2.0)
    return float(np.sum(w * v * u[rows] * u[col]))


from meshgen import box_nnz  # noqa: E402,F401  (structured-box nnz, pinned in test_closed_forms)
