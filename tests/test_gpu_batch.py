"""Batched builds on the GPU (through the C ABI): each mesh of a batch against the FP64
oracle run on that mesh alone, graph capture and replay, data errors, and sampled meshes
of the 256-brick workload.
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import meshgen
import oracle
import paper_1501_04784_amd as kb
from tests.gpu_common import TOL, say
from tests.helpers import scaled_error

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # collected on CPU only when -m gpu is asked for explicitly
    pytest.skip("no GPU", allow_module_level=True)


def small_batch(elem: int, n_mesh: int, seed: int, hi: int = 5):
    """Boxes with cells per axis in U{1..hi}, random numbering, plus an empty mesh."""
    rng = np.random.default_rng(seed)
    out = []
    for m in range(n_mesh):
        nx, ny, nz = (int(v) for v in rng.integers(1, hi + 1, size=3))
        out.append(meshgen.box_mesh(elem, nx, ny, nz, h=1.0 / 8, jitter=0.2, coef=(1e-2, 1e2),
                                    permute_nodes=bool(m % 2), permute_elems=bool(m % 3 == 0), seed=seed * 100 + m))
    empty = meshgen.Mesh(elem, np.zeros((0, elem), np.int32), np.zeros((0, 3)), np.zeros(0))
    return out[: n_mesh // 2] + [empty] + out[n_mesh // 2:]


def as_tuples(meshes):
    return [(m.conn, m.coords, m.coef) for m in meshes]


def check_against_oracle(meshes, results, prec):
    worst = 0.0
    for m, r in zip(meshes, results):
        rp, col = r.row_ptr.cpu().numpy(), r.col_idx.cpu().numpy()
        val = r.vals.cpu().numpy().astype(np.float64)
        if m.n_elem == 0:
            assert rp.tolist() == [0] * (m.n_node + 1) and len(col) == 0
            continue
        orp, ocol, oval, oflags = oracle.build_mesh(m)
        assert oflags == 0
        np.testing.assert_array_equal(rp, orp)
        np.testing.assert_array_equal(col, ocol)
        worst = max(worst, scaled_error(orp, ocol, val, oval))
    return worst


@pytest.mark.parametrize("prec", ["fp64", "fp32fb64"])
@pytest.mark.parametrize("elem", [8, 4])
def test_batch_parity(elem, prec):
    meshes = small_batch(elem, 12, seed=7 + elem)
    say(f"[batch] elem={elem} {prec} meshes={len(meshes)} nel={sum(m.n_elem for m in meshes)}")
    res = kb.build_lower_csr_batched(as_tuples(meshes), elem, prec=prec)
    assert len(res) == len(meshes)
    err = check_against_oracle(meshes, res, prec)
    say(f"  worst scaled error {err:.3e}")
    assert err <= TOL[prec]


def test_batch_equals_single_builds():
    """Each mesh's batched CSR carries the same pattern as its own build, and values equal
    to the last bit (exact sums at a common scale round identically here)."""
    meshes = small_batch(8, 6, seed=3)
    res = kb.build_lower_csr_batched(as_tuples(meshes), 8, prec="fp64")
    for m, r in zip(meshes, res):
        if m.n_elem == 0:
            continue
        d = torch.device("cuda:0")
        one = kb.build_lower_csr(torch.from_numpy(m.conn).to(d), torch.from_numpy(m.coords).to(d),
                                 torch.from_numpy(m.coef).to(d), 8, prec="fp64")
        assert torch.equal(one.row_ptr.cpu(), r.row_ptr.cpu())
        assert torch.equal(one.col_idx.cpu(), r.col_idx.cpu())
        np.testing.assert_allclose(one.vals.cpu().numpy(), r.vals.cpu().numpy(), rtol=0, atol=1e-13 *
                                   float(one.vals.abs().max()))


def test_batch_graph_capture_replays():
    """The batched build enqueues no host synchronisation and no memset: it is captured
    in a HIP graph and replayed; every replay matches the eager result bit for bit."""
    meshes = small_batch(8, 8, seed=11)
    batch = kb.pack_batch(as_tuples(meshes), 8)
    b = kb.BatchBuilder(batch, prec="fp32fb64")
    b.run()
    eager = [(r.row_ptr.clone(), r.col_idx.clone(), r.vals.clone()) for r in b.results()]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        b.run()  # warm the launch path on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        b.run()
    for rep in range(3):
        b.col_idx.fill_(-7)
        b.vals.fill_(float("nan"))
        b.row_ptr.fill_(-7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = b.results()
        for (rp, col, val), r in zip(eager, got):
            assert torch.equal(rp, r.row_ptr) and torch.equal(col, r.col_idx)
            assert torch.equal(val, r.vals), f"replay {rep}"
        _ = torch.ones(1 << 20, device="cuda").sum().item()  # eager work between replays



def test_batch_with_heavy_rows_and_graph_replay():
    """A batch holding two fans among small tet boxes: a centre-last fan of 150,000 tets
    (a row of 450,001 entries whose diagonal is summed by several workgroups) and a
    centre-first one.  Each mesh's CSR has its own build's pattern and values to 1e-13 of
    the largest (the batch sums at one common scale); the batched build captured in a
    HIP graph replays to the eager result bit for bit, the heavy path included."""
    meshes = [meshgen.box_mesh(4, 3, jitter=0.2, coef=(0.5, 2.0), seed=1), meshgen.fan_mesh(150000, True, seed=2),
              meshgen.box_mesh(4, 4, 3, 2, jitter=0.2, seed=4), meshgen.fan_mesh(3000, False, seed=5)]
    say(f"[batch-heavy] meshes={len(meshes)} nel={sum(m.n_elem for m in meshes)}")
    batch = kb.pack_batch(as_tuples(meshes), 4)
    b = kb.BatchBuilder(batch, prec="fp64")
    b.run()
    eager = [(r.row_ptr.clone(), r.col_idx.clone(), r.vals.clone()) for r in b.results()]
    d = torch.device("cuda:0")
    for m, (rp, col, val) in zip(meshes, eager):
        one = kb.build_lower_csr(torch.from_numpy(m.conn).to(d), torch.from_numpy(m.coords).to(d),
                                 torch.from_numpy(m.coef).to(d), 4, prec="fp64")
        assert torch.equal(one.row_ptr, rp) and torch.equal(one.col_idx, col)
        np.testing.assert_allclose(one.vals.cpu().numpy(), val.cpu().numpy(), rtol=0,
                                   atol=1e-13 * float(one.vals.abs().max()))
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        b.run()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        b.run()
    for rep in range(3):
        b.col_idx.fill_(-7)
        b.vals.fill_(float("nan"))
        b.row_ptr.fill_(-7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for (rp, col, val), r in zip(eager, b.results()):
            assert torch.equal(rp, r.row_ptr) and torch.equal(col, r.col_idx)
            assert torch.equal(val, r.vals), f"replay {rep}"
        _ = torch.ones(1 << 20, device="cuda").sum().item()  # eager work between replays

def test_batch_local_id_out_of_range_is_flagged():
    meshes = small_batch(4, 4, seed=5)
    bad = meshes[1]
    conn = bad.conn.copy()
    conn[0, 0] = bad.n_node  # valid in the batch's global numbering, not in its mesh
    meshes[1] = meshgen.Mesh(4, conn, bad.coords, bad.coef)
    res = kb.build_lower_csr_batched(as_tuples(meshes), 4, prec="fp64", check=False)
    assert res[0].flags & kb._lib.KB_F_INDEX


def test_batch_bad_offsets_are_flagged():
    meshes = small_batch(8, 4, seed=9)
    batch = kb.pack_batch(as_tuples(meshes), 8)
    eo = batch.elem_off.clone()
    eo[1], eo[2] = eo[2], eo[1]  # decreasing
    batch = kb.Batch(batch.elem, batch.conn, batch.coords, batch.coef, eo, batch.node_off)
    b = kb.BatchBuilder(batch, prec="fp64")
    b.run()
    with pytest.raises(kb.KBuildError):
        b.results(check=True)


def test_batch_capacity_flag():
    meshes = small_batch(8, 4, seed=2)
    batch = kb.pack_batch(as_tuples(meshes), 8)
    b = kb.BatchBuilder(batch, prec="fp64", cap=10)
    b.run()
    res = b.results(check=False)
    assert res[0].flags & 16
    ref = kb.build_lower_csr_batched(as_tuples(meshes), 8, prec="fp64")
    for r, q in zip(res, ref):  # row pointers are still written
        assert torch.equal(r.row_ptr.cpu(), q.row_ptr.cpu())


def test_batch_256_bricks_sampled():
    """The 256-brick workload (about 11.9M elements): every mesh's nnz and row count, and
    eight meshes in full against the oracle."""
    meshes = meshgen.config4_batch()
    say(f"[batch-256] nel={sum(m.n_elem for m in meshes)}")
    res = kb.build_lower_csr_batched(as_tuples(meshes), 8, prec="fp32fb64")
    for m, r in zip(meshes, res):
        # lower nnz of a structured brick box: the nodes, plus every node pair sharing a
        # brick (axis edges, two diagonals per face, four body diagonals per cell)
        nx, ny, nz = m.meta["nx"], m.meta["ny"], m.meta["nz"]
        X, Y, Z = nx + 1, ny + 1, nz + 1
        pairs = nx * Y * Z + X * ny * Z + X * Y * nz + 2 * (nx * ny * Z + nx * Y * nz + X * ny * nz) + 4 * nx * ny * nz
        assert r.row_ptr.numel() == m.n_node + 1
        assert r.nnz == X * Y * Z + pairs
    rng = np.random.default_rng(0)
    pick = sorted(rng.choice(len(meshes), size=8, replace=False).tolist())
    err = check_against_oracle([meshes[i] for i in pick], [res[i] for i in pick], "fp32fb64")
    say(f"  sampled worst scaled error {err:.3e}")
    assert err <= TOL["fp32fb64"]


@pytest.mark.parametrize("case", ["overshoot", "decreasing"])
def test_batch_bad_node_offsets_stay_in_bounds(case):
    """Node offsets that overshoot the node count or decrease: flagged (KB_F_INDEX), and
    every output is written inside its buffer (row pointers and entry offsets zeroed)."""
    meshes = small_batch(8, 4, seed=9)
    batch = kb.pack_batch(as_tuples(meshes), 8)
    no = batch.node_off.clone()
    n_node = int(batch.coords.shape[0])
    if case == "overshoot":
        no[1] = n_node + 10  # then decreasing back to the total
    else:
        no[2] = max(int(no[1]) - 3, 0)
    batch = kb.Batch(batch.elem, batch.conn, batch.coords, batch.coef, batch.elem_off, no)
    b = kb.BatchBuilder(batch, prec="fp64")
    b.row_ptr.fill_(-7)
    b.nnz_off.fill_(-7)
    b.run()
    torch.cuda.synchronize()
    assert (int(b.status[0].item()) & kb._lib.KB_F_INDEX) != 0
    assert int(b.row_ptr.abs().sum().item()) == 0
    assert int(b.nnz_off.abs().sum().item()) == 0
    with pytest.raises(kb.KBuildError):
        b.results(check=True)


def test_autotune_batch_valid_cached_and_bit_equal(tmp_path):
    """The tuning search on a small batch: its choice is valid for the shape, is stored in
    the JSON cache and read back from it, and builds the batch bit for bit as the
    built-in choice does (every candidate runs the same kernels on the same inputs)."""
    meshes = small_batch(8, 10, seed=21, hi=8)
    batch = kb.pack_batch(as_tuples(meshes), 8, "cuda")
    cache = str(tmp_path / "tuning.json")
    t, entry = kb.tune_batch(batch, "fp32fb64", cache_path=cache)
    say(f"[autotune] chose {t} in {entry['ms']:.3f} ms (built-in {entry['default_ms']:.3f} ms, "
        f"{entry['candidates_timed']} candidates timed)")
    assert entry["source"] == "search" and entry["candidates_timed"] >= 4
    assert entry["ms"] <= entry["default_ms"]
    kb.plan_batched(8, batch.n_mesh, batch.conn.shape[0], batch.coords.shape[0], "fp32fb64", t)  # valid
    tuned = kb.BatchBuilder(batch, "fp32fb64", "auto", tune_cache=cache)
    assert tuned.tune_entry["source"] == "cache" and tuned.tuning == t
    base = kb.BatchBuilder(batch, "fp32fb64")
    tuned.run()
    base.run()
    rt, rb = tuned.results(), base.results()
    assert torch.equal(tuned.nnz_off, base.nnz_off)
    for a, b in zip(rt, rb):
        assert torch.equal(a.row_ptr, b.row_ptr) and torch.equal(a.col_idx, b.col_idx)
        assert torch.equal(a.vals.view(torch.int32), b.vals.view(torch.int32))
    err = check_against_oracle(meshes, rt, "fp32fb64")
    assert err <= TOL["fp32fb64"]
