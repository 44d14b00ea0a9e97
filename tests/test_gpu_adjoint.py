"""Adjoint on the GPU (through the C ABI and the autograd function) against the FP64
oracle's adjoint, which is pinned separately (finite differences of an independent
dense route, invariances).  Tolerance: max |g_gpu - g_oracle| <= 1e-12 * max |g_oracle|
(both FP64; the node sums are exact on the GPU and sequential in the oracle).
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import meshgen
import oracle
import paper_1501_04784_amd as kb
from tests.gpu_common import say, to_dev

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # collected on CPU only when -m gpu is asked for explicitly
    pytest.skip("no GPU", allow_module_level=True)

TOL = 1e-12


def meshes():
    return {
        "hex_c5_small": meshgen.config_mesh(5, n=9),
        "hex_perm": meshgen.box_mesh(8, 7, 5, 6, jitter=0.25, coef=(1e-2, 1e2), permute_nodes=True,
                                     permute_elems=True, seed=31),
        "tet_perm": meshgen.box_mesh(4, 6, 7, 5, jitter=0.2, coef=(1e-3, 1e3), permute_nodes=True,
                                     permute_elems=True, seed=32),
        "tet_single": meshgen.Mesh(4, np.array([[0, 1, 2, 3]], np.int32),
                                   np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], float), np.array([1.5])),
    }


MESHES = meshes()


def rel_err(a, b):
    s = max(float(np.abs(b).max()), 1e-300)
    return float(np.abs(a - b).max()) / s


def run_both(m, seed=0):
    conn, coords, coef = to_dev(m)
    r = kb.build_lower_csr(conn, coords, coef, m.elem, prec="fp64")
    rp, col = r.row_ptr.clone(), r.col_idx.clone()
    w = torch.from_numpy(np.random.default_rng(seed).standard_normal(r.nnz)).to(conn.device)
    gc, gx = kb.adjoint_lower(conn, coords, coef, m.elem, rp, col, w)
    ogc, ogx, f = oracle.adjoint_lower(m, rp.cpu().numpy(), col.cpu().numpy(), w.cpu().numpy())
    assert f == 0
    return gc.cpu().numpy(), gx.cpu().numpy(), ogc, ogx


@pytest.mark.parametrize("name", sorted(MESHES))
def test_adjoint_parity(name):
    m = MESHES[name]
    say(f"[adjoint] {name} nel={m.n_elem}")
    gc, gx, ogc, ogx = run_both(m)
    ec, ex = rel_err(gc, ogc), rel_err(gx, ogx)
    say(f"  dL/dc {ec:.2e}  dL/dX {ex:.2e}")
    assert ec <= TOL and ex <= TOL


def test_adjoint_bitwise_deterministic():
    m = MESHES["tet_perm"]
    a = run_both(m, seed=4)
    b = run_both(m, seed=4)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_reusable_adjoint_context():
    """AdjointBuilder: the same buffers over several calls, with different weights and a
    stale status from a flagged call in between, give the one-shot results bit for bit."""
    m = MESHES["hex_perm"]
    conn, coords, coef = to_dev(m)
    r = kb.build_lower_csr(conn, coords, coef, m.elem, prec="fp64")
    rp, col = r.row_ptr.clone(), r.col_idx.clone()
    a = kb.AdjointBuilder(m.elem, m.n_elem, m.n_node, device=conn.device)
    ws0 = a.ws.data_ptr()
    for seed in (1, 2):
        w = torch.from_numpy(np.random.default_rng(seed).standard_normal(r.nnz)).to(conn.device)
        a.run(conn, coords, coef, rp, col, w)
        gc, gx = (t.clone() for t in a.result())
        ref = kb.adjoint_lower(conn, coords, coef, m.elem, rp, col, w)
        assert torch.equal(gc, ref[0]) and torch.equal(gx, ref[1])
        if seed == 1:  # a flagged call: its status must not leak into the next one
            bad = conn.clone()
            bad[0, 0] = m.n_node
            a.run(bad, coords, coef, rp, col, w)
            with pytest.raises(kb.KBuildError):
                a.result()
    assert a.ws.data_ptr() == ws0
    with pytest.raises(ValueError):
        a.run(conn[:-1], coords, coef[:-1], rp, col, w)


def test_autograd_function():
    m = MESHES["hex_perm"]
    conn, coords, coef = to_dev(m)
    coords = coords.clone().requires_grad_(True)
    coef = coef.clone().requires_grad_(True)
    vals, rp, col = kb.lower_csr_values(coords, coef, conn, m.elem)
    w = torch.from_numpy(np.random.default_rng(9).standard_normal(vals.numel())).to(vals.device)
    loss = (w * vals).sum()
    loss.backward()
    ogc, ogx, f = oracle.adjoint_lower(m, rp.cpu().numpy(), col.cpu().numpy(), w.cpu().numpy())
    assert rel_err(coef.grad.cpu().numpy(), ogc) <= TOL
    assert rel_err(coords.grad.cpu().numpy(), ogx) <= TOL
    # the loss itself matches the oracle's K
    orp, ocol, oval, _ = oracle.build_mesh(m)
    assert abs(loss.item() - float(w.cpu().numpy() @ oval)) <= 1e-12 * float(np.abs(w.cpu().numpy() * oval).sum())


def test_pattern_mismatch_is_flagged():
    m = MESHES["tet_perm"]
    conn, coords, coef = to_dev(m)
    r = kb.build_lower_csr(conn, coords, coef, m.elem, prec="fp64")
    col = r.col_idx.clone()
    col[-1] = col[-1] - 1  # the last row loses its diagonal
    w = torch.ones(r.nnz, dtype=torch.float64, device=conn.device)
    with pytest.raises(kb.KBuildError):
        kb.adjoint_lower(conn, coords, coef, m.elem, r.row_ptr, col, w)


def test_adjoint_c5_full():
    """64^3 bricks (262,144 elements) with the seeded N(0,1) weights of the workload."""
    m = meshgen.config_mesh(5)
    conn, coords, coef = to_dev(m)
    r = kb.build_lower_csr(conn, coords, coef, m.elem, prec="fp64")
    assert r.nnz == 3731841
    w = torch.from_numpy(meshgen.loss_weights(r.nnz)).to(conn.device)
    gc, gx = kb.adjoint_lower(conn, coords, coef, m.elem, r.row_ptr, r.col_idx, w)
    ogc, ogx, f = oracle.adjoint_lower(m, r.row_ptr.cpu().numpy(), r.col_idx.cpu().numpy(), w.cpu().numpy())
    ec, ex = rel_err(gc.cpu().numpy(), ogc), rel_err(gx.cpu().numpy(), ogx)
    say(f"[adjoint-c5] dL/dc {ec:.2e}  dL/dX {ex:.2e}")
    assert ec <= TOL and ex <= TOL


def test_degenerate_element_is_flagged():
    """Two tets sharing a face, the second flat (its fourth node in the shared face,
    at coordinates exact in binary so that det = 0 exactly).  The adjoint flags it
    (inverted, non-finite) and leaves its node contributions out; the first element's
    own gradients still match the oracle."""
    X = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [0.25, 0.25, 0.5]], float)
    m = meshgen.Mesh(4, np.array([[0, 1, 2, 3], [1, 2, 3, 4]], np.int32), X, np.array([1.5, 0.5]))
    conn, coords, coef = to_dev(m)
    allow = kb._lib.KB_F_INVERTED | kb._lib.KB_F_NONFINITE
    r = kb.build_lower_csr(conn, coords, coef, 4, prec="fp64", check=False)
    w = torch.from_numpy(np.random.default_rng(3).standard_normal(r.nnz)).to(conn.device)
    a = kb.AdjointBuilder(4, 2, 5, device=conn.device)
    a.run(conn, coords, coef, r.row_ptr, r.col_idx, w)
    gc, gx = a.result(check=False)
    flags = int(a.status[0].item()) & 0xFFFFFFFF
    assert flags & kb._lib.KB_F_INVERTED and flags & kb._lib.KB_F_NONFINITE
    assert flags & ~allow == 0
    assert bool(torch.isfinite(gx).all())  # the flat element's contributions are dropped
    ogc, ogx, _ = oracle.adjoint_lower(m, r.row_ptr.cpu().numpy(), r.col_idx.cpu().numpy(), w.cpu().numpy())
    assert abs(float(gc[0]) - ogc[0]) <= TOL * abs(ogc[0])
    # node 0 touches only the first element
    assert float((gx[0].cpu() - torch.from_numpy(ogx[0])).abs().max()) <= TOL * float(np.abs(ogx[0]).max())
    with pytest.raises(kb.KBuildError):
        a.result(check=True)


def test_row_pointers_outside_the_pattern_are_flagged():
    """A row pointer beyond the pattern's length is confined by nnz: index flag, no read
    outside col_idx / w.  Wrongly typed or sized row pointers are refused on the host."""
    m = MESHES["tet_perm"]
    conn, coords, coef = to_dev(m)
    r = kb.build_lower_csr(conn, coords, coef, m.elem, prec="fp64")
    rp = r.row_ptr.clone()
    rp[-1] = r.nnz + 1000  # the last row now reaches past col_idx
    w = torch.ones(r.nnz, dtype=torch.float64, device=conn.device)
    with pytest.raises(kb.KBuildError):
        kb.adjoint_lower(conn, coords, coef, m.elem, rp, r.col_idx, w)
    with pytest.raises(ValueError):
        kb.adjoint_lower(conn, coords, coef, m.elem, r.row_ptr.long(), r.col_idx, w)
    with pytest.raises(ValueError):
        kb.adjoint_lower(conn, coords, coef, m.elem, r.row_ptr[:-1], r.col_idx, w)
