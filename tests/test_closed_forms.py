"""The closed-form nnz of structured boxes (used by the full-size GPU checks) against the
oracle's pattern on small boxes of both element types."""
from __future__ import annotations

import pytest

import meshgen
import oracle
from tests.helpers import box_nnz


@pytest.mark.parametrize("elem", [8, 4])
@pytest.mark.parametrize("dims", [(1, 1, 1), (2, 3, 4), (5, 1, 2), (4, 4, 4)])
def test_box_nnz_closed_form(elem, dims):
    m = meshgen.box_mesh(elem, *dims, jitter=0.1, permute_nodes=True, permute_elems=True, seed=sum(dims))
    rp, col, val, f = oracle.build_mesh(m)
    assert f == 0
    assert len(col) == box_nnz(elem, *dims)


def test_box_nnz_matches_the_workload_sizes():
    # hex 100^3 and Kuhn tet 6 x 150^3 (the two single-mesh workloads)
    assert box_nnz(8, 100, 100, 100) == 14_150_601
    assert box_nnz(4, 150, 150, 150) == 27_270_901
