"""Stream and graph behaviour of the builds (through the C ABI): the single-mesh,
grouped and several-DOF builds enqueue no host synchronisation and no memset, so each is
captured in a HIP graph and replayed; every replay (with the program's own eager work
and synchronisations between replays) matches the eager result bit for bit.  Two builds
on two streams at once, each with its own workspace, give their own results."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import meshgen
import paper_1501_04784_amd as kb
from tests.gpu_common import say, to_dev
from tests.helpers import box_nnz

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # collected on CPU only when -m gpu is asked for explicitly
    pytest.skip("no GPU", allow_module_level=True)


def outputs(b):
    return b.row_ptr, b.col_idx, b.vals


def replay_matches(b, run):
    """Capture run() in a graph, replay it three times against the eager result."""
    run()
    r = b.result()
    n = r.nnz  # entries past nnz are not written
    eager = [b.row_ptr.clone(), b.col_idx[:n].clone(), b.vals[:n].clone()]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        run()  # warm the launch path on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        run()
    for rep in range(3):
        for t in outputs(b):
            t.fill_(-7 if t.dtype == torch.int32 else float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = [b.row_ptr, b.col_idx[:n], b.vals[:n]]
        for a, e in zip(got, eager):
            assert torch.equal(a, e), f"replay {rep}"
        _ = torch.ones(1 << 20, device="cuda").sum().item()  # eager work between replays
    return r


@pytest.mark.parametrize("prec", ["fp32fb64", "fp64"])
@pytest.mark.parametrize("elem", [4, 8])
def test_single_build_graph_replays(elem, prec):
    m = meshgen.config_mesh(3 if elem == 4 else 2, n=12)
    conn, coords, coef = to_dev(m)
    b = kb.Builder(elem, m.n_elem, m.n_node, prec=prec)
    r = replay_matches(b, lambda: b.run(conn, coords, coef))
    say(f"[graph] elem={elem} {prec} nnz={r.nnz}")


def test_grouped_build_graph_replays():
    m = meshgen.config_mesh(3, n=10)
    conn, coords, coef = to_dev(m)
    b = kb.GroupedBuilder(4, m.n_elem, m.n_node, 1500, box_nnz(4, 10, 10, 10), prec="fp32fb64")
    replay_matches(b, lambda: b.run(conn, coords, coef))


def test_dof_assembly_graph_replays():
    m = meshgen.config_mesh(2, n=8)
    conn, _, _ = to_dev(m)
    klow = torch.from_numpy(meshgen.element_matrices(m.n_elem, 24, 3)).to(conn.device)
    b = kb.Builder(8, m.n_elem, m.n_node, prec="fp64", dof=3)
    replay_matches(b, lambda: b.run(conn, None, None, klow=klow))


def test_two_streams_at_once():
    ma, mb = meshgen.config_mesh(3, n=14), meshgen.config_mesh(2, n=20)
    da, db = to_dev(ma), to_dev(mb)
    ba = kb.Builder(4, ma.n_elem, ma.n_node, prec="fp32fb64")
    bb = kb.Builder(8, mb.n_elem, mb.n_node, prec="fp32fb64")
    ra_ref = kb.build_lower_csr(*da, 4, prec="fp32fb64")
    rb_ref = kb.build_lower_csr(*db, 8, prec="fp32fb64")
    torch.cuda.synchronize()
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    for _ in range(3):
        with torch.cuda.stream(sa):
            ba.run(*da)
        with torch.cuda.stream(sb):
            bb.run(*db)
    torch.cuda.synchronize()
    ra, rb = ba.result(), bb.result()
    for r, ref in ((ra, ra_ref), (rb, rb_ref)):
        assert r.nnz == ref.nnz
        assert torch.equal(r.row_ptr, ref.row_ptr) and torch.equal(r.col_idx, ref.col_idx)
        assert torch.equal(r.vals, ref.vals)
    assert np.isfinite(ra.vals.cpu().numpy()).all()
