"""The all-cores timing harness of the oracle (oracle/timing_par.c) builds the same
matrix as the single-threaded oracle: the same pattern, values equal to rounding (only
the order in which duplicates are summed differs), the same data flags; with any
thread count."""
from __future__ import annotations

import numpy as np
import pytest

import meshgen
import oracle
from tests.helpers import scaled_error


@pytest.mark.parametrize("threads", [0, 1, 3, 8])
@pytest.mark.parametrize("cid,n", [(3, 12), (2, 9), (1, None)])
def test_par_harness_matches_oracle(cid, n, threads):
    m = meshgen.config_mesh(cid, n=n)
    a = oracle.build_mesh(m)
    b = oracle.par_build_mesh(m, threads)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])
    assert scaled_error(a[0], a[1], b[2], a[2]) <= 1e-14
    assert a[3] == b[3] == 0


def test_par_harness_flags_and_skips_bad_elements():
    m = meshgen.box_mesh(4, 4, jitter=0.1, permute_nodes=True, seed=5)
    conn = m.conn.copy()
    conn[3, 1] = m.n_node  # index error: the element is left out
    conn[7, 2] = conn[7, 0]  # repeated node: left out
    bad = meshgen.Mesh(4, conn, m.coords, m.coef)
    a = oracle.build_mesh(bad)
    b = oracle.par_build_mesh(bad, 4)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])
    assert scaled_error(a[0], a[1], b[2], a[2]) <= 1e-14
    assert a[3] == b[3] == 3


def test_par_threads_positive():
    assert oracle.par_threads() >= 1
