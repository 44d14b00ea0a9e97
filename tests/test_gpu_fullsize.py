"""The single-mesh workloads at full size, in the launch configuration the benchmark
times (default tuning, its precision): the Kuhn tet box 6 x 150^3 (20,250,000 elements),
the brick box 100^3 (1,000,000 elements) and the 300^3 brick cube of Table 2.

* the pattern: nnz against the closed form of the box, columns ascending within each
  row, the diagonal last and positive;
* sampled rows against the FP64 oracle, which computes selected rows one by one from
  all elements: exact pattern, values within the precision's scaled tolerance;
* a property of the whole matrix: every row of the full symmetric K sums to zero
  (constants are in the kernel of the Poisson operator), up to the precision.
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import meshgen
import oracle
import paper_1501_04784_amd as kb
from tests.gpu_common import TOL, say, to_dev
from tests.helpers import box_nnz

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # collected on CPU only when -m gpu is asked for explicitly
    pytest.skip("no GPU", allow_module_level=True)

# relative row-sum bound of the full symmetric K, per precision
ROWSUM = {"fp64": 1e-12, "fp32fb64": 2e-5, "fp32": 2e-5}
_MESHES = {}


def workload(cid):
    if cid not in _MESHES:
        _MESHES.clear()
        _MESHES[cid] = meshgen.config_mesh(cid)
    return _MESHES[cid]


def check_pattern(m, r, dims):
    rp = r.row_ptr.long()
    n = m.n_node
    assert r.nnz == box_nnz(m.elem, *dims)
    assert int(rp[0]) == 0 and int(rp[-1]) == r.nnz
    lens = rp[1:] - rp[:-1]
    assert bool((lens >= 1).all())
    col = r.col_idx.long()
    rows = torch.repeat_interleave(torch.arange(n, device=rp.device), lens)
    # ascending columns within rows (a row boundary may step down), diagonal last and positive
    step_ok = (col[1:] > col[:-1]) | (rows[1:] != rows[:-1])
    assert bool(step_ok.all())
    last = rp[1:] - 1
    assert bool((col[last] == torch.arange(n, device=rp.device)).all())
    assert bool((col <= rows).all())
    assert bool((r.vals[last] > 0).all())
    return rows, col


def check_row_sums(r, rows, col, prec):
    v = r.vals.double()
    n = r.row_ptr.numel() - 1
    s = torch.zeros(n, dtype=torch.float64, device=v.device).index_add_(0, rows, v)
    a = torch.zeros(n, dtype=torch.float64, device=v.device).index_add_(0, rows, v.abs())
    off = rows != col
    s.index_add_(0, col[off], v[off])
    a.index_add_(0, col[off], v[off].abs())
    worst = float((s.abs() / a).max())
    say(f"  worst relative row sum {worst:.2e}")
    assert worst <= ROWSUM[prec]


def check_sampled_rows(m, r, prec, n_sample=1500, seed=0):
    rp = r.row_ptr.cpu().numpy()
    col = r.col_idx.cpu().numpy()
    val = r.vals.cpu().numpy().astype(np.float64)
    lens = np.diff(rp)
    rng = np.random.default_rng(seed)
    pick = set(rng.choice(m.n_node, size=n_sample, replace=False).tolist())
    pick |= {0, m.n_node - 1, int(np.argmax(lens))}
    pick = np.array(sorted(pick), np.int32)
    # the oracle's rows for the picked rows and for every column they touch (their diagonals scale)
    need = np.unique(np.concatenate([pick, *[col[rp[i]:rp[i + 1]] for i in pick]])).astype(np.int32)
    optr, ocol, oval = oracle.rows_lower(m.elem, m.conn, m.coords, m.coef, need)
    diag = {}
    for k, i in enumerate(need):
        assert ocol[optr[k + 1] - 1] == i
        diag[int(i)] = oval[optr[k + 1] - 1]
    where = {int(i): k for k, i in enumerate(need)}
    worst = 0.0
    for i in pick:
        k = where[int(i)]
        oc, ov = ocol[optr[k]:optr[k + 1]], oval[optr[k]:optr[k + 1]]
        gc, gv = col[rp[i]:rp[i + 1]], val[rp[i]:rp[i + 1]]
        np.testing.assert_array_equal(gc, oc)
        scale = np.sqrt(np.abs(diag[int(i)] * np.array([diag[int(j)] for j in oc])))
        worst = max(worst, float(np.max(np.abs(gv - ov) / scale)))
    say(f"  {len(pick)} sampled rows, worst scaled error {worst:.2e}")
    assert worst <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp32fb64", "fp64"])
def test_tet_150_full_size(prec):
    m = workload(3)
    say(f"[full] tet 6x150^3 {prec} nel={m.n_elem} nn={m.n_node}")
    r = kb.build_lower_csr(*to_dev(m), m.elem, prec=prec)
    say(f"  nnz={r.nnz} fallback={r.n_fallback}")
    rows, col = check_pattern(m, r, (150, 150, 150))
    check_row_sums(r, rows, col, prec)
    check_sampled_rows(m, r, prec)


def test_brick_100_full_size():
    m = workload(2)
    say(f"[full] hex 100^3 fp32fb64 nel={m.n_elem} nn={m.n_node}")
    r = kb.build_lower_csr(*to_dev(m), m.elem, prec="fp32fb64")
    rows, col = check_pattern(m, r, (100, 100, 100))
    check_row_sums(r, rows, col, "fp32fb64")
    check_sampled_rows(m, r, "fp32fb64")


def test_brick_300_table2_full_size():
    """The largest mesh of the paper's Table 2 (27,000,000 undistorted unit-cube bricks,
    27,270,901 nodes), FP64 as the paper's values: nnz, rows against the oracle, row sums."""
    m = workload(7)
    say(f"[full] hex 300^3 fp64 nel={m.n_elem} nn={m.n_node}")
    r = kb.build_lower_csr(*to_dev(m), m.elem, prec="fp64")
    rows, col = check_pattern(m, r, (300, 300, 300))
    check_row_sums(r, rows, col, "fp64")
    del rows, col
    check_sampled_rows(m, r, "fp64", n_sample=800)
