"""Parity of the HIP path (through the C ABI) with the FP64 oracle, on the GPU.

Pattern (row_ptr, col_idx) must match bit for bit; values within the scaled
tolerance max |dK_ij| / sqrt(K_ii K_jj) of 1e-12 (FP64) and 5e-6 (FP32 with FP64
fallback).  Sizes are chosen so that the oracle finishes in about a second while
the launch still spans many workgroups and ends in a ragged tail.
"""
from __future__ import annotations

import math

import numpy as np
import pytest
import torch

import meshgen
import oracle
import paper_1501_04784_amd as kb
from tests.gpu_common import TOL, elem_scaled_error, gpu_build, np_csr, say, to_dev
from tests.helpers import scaled_error

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # collected on CPU only when -m gpu is asked for explicitly
    pytest.skip("no GPU", allow_module_level=True)

PRECS = ["fp64", "fp32fb64", "fp32"]


def small_meshes():
    return {
        "c1_hex10": meshgen.config_mesh(1),
        "c2_hex13": meshgen.config_mesh(2, n=13),
        "c3_tet9": meshgen.config_mesh(3, n=9),
        "c5_hex16": meshgen.config_mesh(5, n=16),
        "tet_box_7x5x3": meshgen.box_mesh(4, 7, 5, 3, jitter=0.2, coef=(0.1, 10), permute_nodes=True,
                                          permute_elems=True, seed=21),
        "hex_box_1x1x1": meshgen.box_mesh(8, 1, jitter=0.0, coef=2.0, seed=0),
        "tet_single": meshgen.Mesh(4, np.array([[0, 1, 2, 3]], np.int32),
                                   np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], float), np.array([1.5])),
    }


MESHES = small_meshes()


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("name", sorted(MESHES))
def test_integrate_parity(name, prec):
    m = MESHES[name]
    say(f"[integrate] {name} {prec} nel={m.n_elem}")
    conn, coords, coef = to_dev(m)
    k, status = kb.integrate_lower(conn, coords, coef, m.elem, prec=prec)
    kref, flags = oracle.integrate_lower(m.elem, m.conn, m.coords, m.coef)
    assert flags == 0
    err = elem_scaled_error(k.cpu().numpy().astype(np.float64), kref, m.elem)
    say(f"  element scaled error {err:.3e}")
    assert err <= TOL[prec]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("name", sorted(MESHES))
def test_build_parity(name, prec):
    m = MESHES[name]
    say(f"[build] {name} {prec} nel={m.n_elem} nn={m.n_node}")
    r = gpu_build(m, prec)
    rp, col, val = np_csr(r)
    orp, ocol, oval, oflags = oracle.build_mesh(m)
    assert oflags == 0 and r.flags == 0
    np.testing.assert_array_equal(rp, orp)
    np.testing.assert_array_equal(col, ocol)
    err = scaled_error(orp, ocol, val, oval)
    say(f"  nnz={len(col)} scaled error {err:.3e} fallback={r.n_fallback}")
    assert err <= TOL[prec]


@pytest.mark.parametrize("nz", [11, 9])
@pytest.mark.parametrize("op", ["stiffness", "mass"])
@pytest.mark.parametrize("block", [256, 192, 128])
def test_fp64_brick_tiles(block, op, nz):
    """Every FP64 brick pass-1 tile (256 by default, 192 where many buckets crowd the LDS,
    128 the half tile), forced through the tuning, against the oracle: a randomly numbered
    box spanning several tiles with a ragged last one.  Workgroups take two tiles each; the
    two boxes (4807 and 3933 bricks) give every tile size both an odd tile count (a last
    workgroup with one tile) and an even one."""
    m = meshgen.box_mesh(8, 23, 19, nz, jitter=0.25, coef=(0.1, 10), permute_nodes=True, permute_elems=True,
                         seed=77)
    ntiles = -(-m.n_elem // block)
    say(f"[tile] block={block} {op} nel={m.n_elem} tiles={ntiles}")
    conn, coords, coef = to_dev(m)
    r = kb.build_lower_csr(conn, coords, coef, 8, prec="fp64", op=op, tuning=kb.Tuning(block=block))
    rp, col, val = np_csr(r)
    orp, ocol, oval, oflags = (oracle.build_mass_mesh if op == "mass" else oracle.build_mesh)(m)
    assert oflags == 0 and r.flags == 0
    np.testing.assert_array_equal(rp, orp)
    np.testing.assert_array_equal(col, ocol)
    assert scaled_error(orp, ocol, val, oval) <= TOL["fp64"]


@pytest.mark.parametrize("prec", ["fp64", "fp32fb64"])
@pytest.mark.parametrize("elem,n", [(8, 40), (4, 30)])
def test_build_parity_medium(elem, n, prec):
    """64k bricks / 162k tets with random numbering: many row blocks, exact pattern."""
    cid = 2 if elem == 8 else 3
    m = meshgen.config_mesh(cid, n=n)
    say(f"[build-medium] elem={elem} n={n} {prec} nel={m.n_elem}")
    r = gpu_build(m, prec)
    rp, col, val = np_csr(r)
    orp, ocol, oval, _ = oracle.build_mesh(m)
    np.testing.assert_array_equal(rp, orp)
    np.testing.assert_array_equal(col, ocol)
    err = scaled_error(orp, ocol, val, oval)
    say(f"  nnz={len(col)} scaled error {err:.3e} fallback={r.n_fallback}")
    assert err <= TOL[prec]


@pytest.mark.parametrize("elem", [8, 4])
@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 7, 8, 11, 13, 16, 21])
def test_build_parity_size_sweep(elem, n):
    """Many mesh sizes: workspace regions, tiles and buckets take many shapes."""
    m = meshgen.box_mesh(elem, n, n + 1, max(1, n - 1), jitter=0.2, coef=(0.1, 10), permute_nodes=True,
                         permute_elems=True, seed=100 + n)
    r = gpu_build(m, "fp64")
    rp, col, val = np_csr(r)
    orp, ocol, oval, _ = oracle.build_mesh(m)
    np.testing.assert_array_equal(rp, orp)
    np.testing.assert_array_equal(col, ocol)
    assert scaled_error(orp, ocol, val, oval) <= TOL["fp64"]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name", ["c2_hex13", "c3_tet9"])
def test_assemble_parity(name, prec):
    """Assembly alone from the oracle's element values (cast to the value type)."""
    m = MESHES[name]
    kref, _ = oracle.integrate_lower(m.elem, m.conn, m.coords, m.coef)
    dt = torch.float64 if prec == "fp64" else torch.float32
    klow = torch.from_numpy(kref).to(dt).cuda()
    conn = torch.from_numpy(m.conn).cuda()
    r = kb.assemble_lower_csr(conn, m.n_node, klow, m.elem, prec=prec)
    rp, col, val = np_csr(r)
    kin = klow.cpu().numpy().astype(np.float64)
    orp, ocol, oval, _ = oracle.assemble_lower_csr(m.elem, m.conn, m.n_node, kin)
    np.testing.assert_array_equal(rp, orp)
    np.testing.assert_array_equal(col, ocol)
    # same inputs: only summation order and the final rounding differ
    assert scaled_error(orp, ocol, val, oval) <= (1e-15 if prec == "fp64" else 1e-7)


@pytest.mark.parametrize("prec", ["fp64", "fp32fb64"])
def test_bitwise_determinism(prec):
    m = meshgen.config_mesh(3, n=20)
    a = np_csr(gpu_build(m, prec))
    b = np_csr(gpu_build(m, prec))
    for x, y in zip(a, b):
        assert x.tobytes() == y.tobytes()


def renumbered(m, seed):
    """The same mesh with its nodes renumbered and its elements reordered (each element's
    local node order kept): old node i becomes p[i]."""
    rng = np.random.default_rng(seed)
    p = rng.permutation(m.n_node).astype(np.int64)
    q = rng.permutation(m.n_elem)
    coords = np.empty_like(m.coords)
    coords[p] = m.coords
    return meshgen.Mesh(m.elem, p[m.conn[q]].astype(np.int32), coords, m.coef[q]), p


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("elem,dims", [(8, (23, 17, 11)), (4, (13, 11, 9)), (8, (60, 60, 60))])
def test_renumbering_permutes_k_bitwise(elem, dims, prec):
    """Every element value is computed from the same coordinates in the same local order
    and each entry is an exact sum rounded once, so renumbering the nodes of a naturally
    numbered box (and reordering its elements) must permute K bit for bit: entry (i, j)
    moves to (max(p_i, p_j), min(p_i, p_j)), K being symmetric."""
    m = meshgen.box_mesh(elem, *dims, jitter=0.2, coef=(0.1, 10), seed=31)
    mp, p = renumbered(m, 32)
    say(f"[renumber] elem={elem} dims={dims} {prec} nel={m.n_elem}")
    n = m.n_node
    rp, col, _ = np_csr(r0 := gpu_build(m, prec))
    rq, colq, _ = np_csr(r1 := gpu_build(mp, prec))
    val, valq = r0.vals.cpu().numpy(), r1.vals.cpu().numpy()
    a = p[np.repeat(np.arange(n), np.diff(rp))]
    b = p[col.astype(np.int64)]
    key_old = np.maximum(a, b) * n + np.minimum(a, b)
    key_new = np.repeat(np.arange(n, dtype=np.int64), np.diff(rq)) * n + colq.astype(np.int64)
    o, w = np.argsort(key_old, kind="stable"), np.argsort(key_new, kind="stable")
    np.testing.assert_array_equal(key_old[o], key_new[w])
    assert val[o].tobytes() == valq[w].tobytes()


def test_empty_mesh():
    m = meshgen.Mesh(4, np.zeros((0, 4), np.int32), np.zeros((5, 3)), np.zeros(0))
    conn, coords, coef = to_dev(m)
    r = kb.build_lower_csr(conn, coords, coef, 4, prec="fp64")
    assert r.nnz == 0
    assert r.row_ptr.cpu().tolist() == [0] * 6


def test_unused_nodes_have_empty_rows():
    m = meshgen.box_mesh(4, 3, jitter=0.1, seed=9)
    coords = np.vstack([m.coords, np.zeros((4, 3))])  # four nodes no element touches
    m2 = meshgen.Mesh(4, m.conn, coords, m.coef)
    r = gpu_build(m2, "fp64")
    rp, col, val = np_csr(r)
    orp, ocol, oval, _ = oracle.build_mesh(m2)
    np.testing.assert_array_equal(rp, orp)
    assert np.all(np.diff(rp[-5:]) == 0)


def _fan(n_tets, center_last, seed=0):
    """n_tets well-shaped tets sharing one node (meshgen.fan_mesh): its row (centre last)
    or diagonal collects every element."""
    return meshgen.fan_mesh(n_tets, center_last, seed)


def _stars(k, n):
    """k fans of n tets side by side (node ids in blocks of 3 n + 1, each centre last in
    its block; coordinates shifted apart)."""
    fans = [_fan(n, True, seed=s) for s in range(k)]
    nn = fans[0].n_node
    conn = np.concatenate([f.conn + i * nn for i, f in enumerate(fans)]).astype(np.int32)
    X = np.concatenate([f.coords + 10.0 * i for i, f in enumerate(fans)])
    return meshgen.Mesh(4, conn, X, np.concatenate([f.coef for f in fans]))


@pytest.mark.parametrize("n_tets,center_last", [(5000, False), (5000, True), (20000, True), (200000, True),
                                                (1_500_000, True)])
@pytest.mark.parametrize("prec", ["fp64", "fp32fb64"])
def test_heavy_row(n_tets, center_last, prec):
    """A node shared by n elements.  With the centre last, its row holds 3 n + 1 distinct
    entries (more than any LDS hash table: the heavy-sub-bucket kernel); from 20000 tets
    its sub-bucket also exceeds 2^16 pairs and its diagonal sums n pairs over several
    carry rounds; 200000 tets split the row once into leaf ranges, 1.5M tets (4.5M
    columns, more than 2^22) split it twice."""
    m = _fan(n_tets, center_last)
    say(f"[heavy] n={n_tets} centre_last={center_last} {prec}")
    r = gpu_build(m, prec)
    rp, col, val = np_csr(r)
    orp, ocol, oval, _ = oracle.build_mesh(m)
    np.testing.assert_array_equal(rp, orp)
    np.testing.assert_array_equal(col, ocol)
    # the centre's diagonal sums one value per element.  The oracle sums in sequence, so
    # its own rounding error grows to about n * 2^-53 of the sum (2e-11 at 200000 terms,
    # above the FP64 tolerance); that entry is referenced to the correctly rounded sum of
    # the oracle's element values instead (each element's (0, 0) value: the centre is
    # its first node)
    c = m.n_node - 1 if center_last else 0
    klow, _ = oracle.integrate_lower(m.elem, m.conn, m.coords, m.coef)
    oval = oval.copy()
    oval[orp[c + 1] - 1] = math.fsum(klow[:, 0].tolist())
    err = scaled_error(orp, ocol, val, oval)
    say(f"  nnz={len(col):,} scaled error {err:.2e}")
    assert err <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32fb64"])
def test_many_heavy_rows(prec):
    """Ninety-six stars of 3000 tets, each centre numbered last within its star: 96 rows
    of 9001 entries, each in a sub-bucket of its own and past every table, so that as
    many sub-buckets are listed for the heavy path as the many-workgroup split takes
    (64) and more go to the single-workgroup one.  Every entry against the oracle, and
    the same matrix bit for bit on a second build (the list order differs from run to
    run)."""
    k, n = 96, 3000
    m = _stars(k, n)
    nn = m.n_node // k
    say(f"[many-heavy] {k} stars of {n} tets {prec}")
    r = gpu_build(m, prec)
    rp, col, val = np_csr(r)
    again = np_csr(gpu_build(m, prec))
    for x, y in zip((rp, col, val), again):
        assert np.array_equal(x.view(np.uint8), y.view(np.uint8))
    orp, ocol, oval, _ = oracle.build_mesh(m)
    np.testing.assert_array_equal(rp, orp)
    np.testing.assert_array_equal(col, ocol)
    # each centre's diagonal against the correctly rounded sum of its elements' values
    klow, _ = oracle.integrate_lower(m.elem, m.conn, m.coords, m.coef)
    oval = oval.copy()
    for i in range(k):
        c = (i + 1) * nn - 1
        oval[orp[c + 1] - 1] = math.fsum(klow[i * n:(i + 1) * n, 0].tolist())
    err = scaled_error(orp, ocol, val, oval)
    say(f"  nnz={len(col):,} scaled error {err:.2e}")
    assert err <= TOL[prec]



@pytest.mark.parametrize("prec", ["fp64", "fp32fb64"])
def test_one_element_repeated(prec):
    """40,000 copies of one tet over four nodes, each with its own coefficient: ten
    entries, 400,000 pairs in one sub-bucket (past 2^16: the heavy path, with a 2-bit
    column space and one digit per row).  Row 3's 160,000 pairs are more than one
    workgroup sums alone (a big leaf), row 2's 120,000 take two carry rounds.  The build
    against the oracle (each entry referred to the correctly rounded sum of the oracle's
    element values, math.fsum); then the oracle's FP64 element values assembled by the
    library, which must give exactly those correctly rounded sums (no bit of these
    values falls below the fixed-point scale)."""
    n = 40000
    rng = np.random.default_rng(11)
    conn = np.tile(np.arange(4, dtype=np.int32), (n, 1))
    X = np.array([[0.0, 0.0, 0.0], [1.0, 0.1, 0.0], [0.2, 1.1, 0.0], [0.1, 0.2, 0.9]])
    m = meshgen.Mesh(4, conn, X, np.exp(rng.uniform(-2, 2, n)))
    say(f"[repeated] {n} copies of one tet {prec}")
    rp, col, val = np_csr(gpu_build(m, prec))
    np.testing.assert_array_equal(rp, [0, 1, 3, 6, 10])
    np.testing.assert_array_equal(col, [0, 0, 1, 0, 1, 2, 0, 1, 2, 3])
    klow, _ = oracle.integrate_lower(m.elem, m.conn, m.coords, m.coef)
    want = np.array([math.fsum(klow[:, t].tolist()) for t in range(10)])  # lower order = CSR order here
    err = scaled_error(rp, col, val.astype(np.float64), want)
    say(f"  scaled error {err:.2e}")
    assert err <= TOL[prec]
    if prec == "fp64":
        d = torch.device("cuda:0")
        r = kb.assemble_lower_csr(torch.from_numpy(conn).to(d), 4, torch.from_numpy(klow).to(d), 4, prec="fp64")
        got = r.vals[:10].cpu().numpy()
        assert np.array_equal(got.view(np.uint64), want.view(np.uint64)), (got - want) / np.spacing(want)

def test_capacity_flag():
    m = meshgen.config_mesh(1)
    r = gpu_build(m, "fp64", cap=1000, check=False)
    assert r.flags & kb._lib.KB_F_CAPACITY
    assert r.nnz == 15561
    orp = oracle.build_mesh(m)[0]
    np.testing.assert_array_equal(r.row_ptr.cpu().numpy(), orp)


@pytest.mark.parametrize("kind", ["index", "negative", "repeat", "inverted", "nan", "inf_coef"])
def test_data_error_flags(kind):
    m = meshgen.box_mesh(4, 4, jitter=0.1, coef=(0.5, 2.0), permute_nodes=True, seed=5)
    conn, coords, coef = m.conn.copy(), m.coords.copy(), m.coef.copy()
    want = {"index": kb._lib.KB_F_INDEX, "negative": kb._lib.KB_F_INDEX, "repeat": kb._lib.KB_F_REPEAT,
            "inverted": kb._lib.KB_F_INVERTED, "nan": kb._lib.KB_F_NONFINITE, "inf_coef": kb._lib.KB_F_NONFINITE}[kind]
    if kind == "index":
        conn[17, 2] = m.n_node
    elif kind == "negative":
        conn[3, 0] = -5
    elif kind == "repeat":
        conn[8, 3] = conn[8, 1]
    elif kind == "inverted":
        conn[11, [2, 3]] = conn[11, [3, 2]]
    elif kind == "nan":
        coords[conn[4, 2], 0] = np.nan
    else:
        coef[9] = np.inf
    bad = meshgen.Mesh(4, conn, coords, coef)
    for prec in PRECS:
        r = gpu_build(bad, prec, check=False)
        assert r.flags & want, (kind, prec, r.flags)
        oflags = oracle.build_mesh(bad)[3]
        assert oflags & want
        if kind in ("index", "negative", "repeat"):
            # the offending element is excluded, exactly as in the oracle
            orp, ocol, oval, _ = oracle.build_mesh(bad)
            rp, col, val = np_csr(r)
            np.testing.assert_array_equal(rp, orp)
            np.testing.assert_array_equal(col, ocol)
            assert scaled_error(orp, ocol, val, oval) <= TOL[prec]
        with pytest.raises(kb.KBuildError):
            gpu_build(bad, prec, check=True)


def test_fallback_fires_on_distorted_mesh():
    """Heavily distorted bricks trigger the FP64 Jacobian path and stay within tolerance."""
    m = meshgen.box_mesh(8, 10, jitter=0.45, coef=(1e-2, 1e2), permute_nodes=True, seed=13)
    r = gpu_build(m, "fp32fb64", allow_flags=kb._lib.KB_F_INVERTED)
    orp, ocol, oval, _ = oracle.build_mesh(m)
    rp, col, val = np_csr(r)
    np.testing.assert_array_equal(col, ocol)
    say(f"  fallback elements {r.n_fallback} of {m.n_elem}")
    assert r.n_fallback > 0
    assert scaled_error(orp, ocol, val, oval) <= TOL["fp32fb64"]


def test_lower_csr_tensor():
    """The build as torch.sparse_csr_tensor: the same row pointers, columns and values as
    the CSR arrays, int32 indices, usable by torch's sparse products (K x against the
    oracle's matrix)."""
    m = MESHES["c3_tet9"]
    t = kb.lower_csr_tensor(*to_dev(m), m.elem, prec="fp64")
    assert t.layout == torch.sparse_csr and t.shape == (m.n_node, m.n_node)
    assert t.crow_indices().dtype == torch.int32 and t.col_indices().dtype == torch.int32
    orp, ocol, oval, _ = oracle.build_mesh(m)
    np.testing.assert_array_equal(t.crow_indices().cpu().numpy(), orp)
    np.testing.assert_array_equal(t.col_indices().cpu().numpy(), ocol)
    x = np.random.default_rng(1).standard_normal(m.n_node)
    y = (t.to(torch.float64) @ torch.from_numpy(x).cuda()).cpu().numpy()
    rows = np.repeat(np.arange(m.n_node), np.diff(orp))
    ref = np.zeros(m.n_node)
    np.add.at(ref, rows, oval * x[ocol])
    assert np.max(np.abs(y - ref)) <= 1e-12 * np.max(np.abs(ref))
