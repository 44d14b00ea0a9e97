"""Grouped builds (Eq. 10: K as the sum over element groups, each group's sums carried
into the next group's pass) on the GPU, through the C ABI:

* against the single-pass build of the same mesh for many group sizes: identical
  pattern; values within one rounding or the fixed-point truncation (the number of
  bitwise-equal entries is reported);
* against the FP64 oracle; both operators; data errors raised by any group; the
  capacity rule; an empty mesh;
* a Kuhn tet box of 6 x 337^3 = 229,636,518 elements, whose 2,296,365,180 element
  pairs exceed what one pass indexes (2^31), built in two groups: nnz against the
  closed form, sampled rows against the oracle, zero row sums of the whole matrix;
* the groups streamed from pinned host memory (kb_build_lower_csr_group_pass), equal to
  the device-resident grouped build bit for bit;
* the pass-3 table size set by hand, bit for bit the built-in one.
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import meshgen
import oracle
import paper_1501_04784_amd as kb
from tests.gpu_common import TOL, np_csr, say, to_dev
from tests.helpers import box_nnz, scaled_error
from tests.test_gpu_fullsize import check_pattern, check_row_sums, check_sampled_rows

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # collected on CPU only when -m gpu is asked for explicitly
    pytest.skip("no GPU", allow_module_level=True)

MESHES = {
    "tet_c3_n9": lambda: meshgen.config_mesh(3, n=9),     # 4,374 tets, random numbering
    "hex_c2_n13": lambda: meshgen.config_mesh(2, n=13),   # 2,197 bricks, random node numbering
}


def compare_to_single(m, prec, group, op="stiffness"):
    dev = to_dev(m)
    one = kb.build_lower_csr(*dev, m.elem, prec=prec, op=op)
    grp = kb.build_lower_csr_grouped(*dev, m.elem, group, cap=one.nnz, prec=prec, op=op)
    assert grp.nnz == one.nnz
    assert torch.equal(grp.row_ptr, one.row_ptr) and torch.equal(grp.col_idx, one.col_idx)
    a, b = grp.vals.double(), one.vals.double()
    # each pass truncates its values at 2^-F, F from that pass's largest value, so the two
    # routes sum the same values truncated at different scales (the bits of values more
    # than 2^42 below the largest): they agree to within one rounding or a few units of
    # 2^-94 of the largest entry
    eps = 2.0 ** -52 if prec == "fp64" else 2.0 ** -23
    bound = torch.maximum(eps * b.abs(), torch.full_like(b, 2.0 ** -80 * float(b.abs().max())))
    assert bool(((a - b).abs() <= bound).all())
    same = int((grp.vals == one.vals).sum())
    say(f"  group={group}: {same}/{one.nnz} entries bitwise equal to the single pass")
    return grp, one


@pytest.mark.parametrize("prec", ["fp64", "fp32fb64", "fp32"])
@pytest.mark.parametrize("name", sorted(MESHES))
def test_grouped_matches_single_pass(name, prec):
    m = MESHES[name]()
    say(f"[grouped] {name} {prec} nel={m.n_elem}")
    for group in (97, m.n_elem // 3, m.n_elem - 1, m.n_elem, 10 * m.n_elem):
        compare_to_single(m, prec, group)


def test_grouped_one_element_per_group():
    m = meshgen.box_mesh(4, 2, 2, 1, jitter=0.2, coef=(0.5, 2.0), permute_nodes=True, permute_elems=True, seed=3)
    compare_to_single(m, "fp64", 1)


@pytest.mark.parametrize("prec", ["fp64", "fp32fb64"])
def test_grouped_against_the_oracle(prec):
    m = meshgen.config_mesh(3, n=14)
    grp = kb.build_lower_csr_grouped(*to_dev(m), m.elem, 5000, cap=box_nnz(4, 14, 14, 14), prec=prec)
    rp, col, val = np_csr(grp)
    orp, ocol, oval, _ = oracle.build_mesh(m)
    np.testing.assert_array_equal(rp, orp)
    np.testing.assert_array_equal(col, ocol)
    assert scaled_error(orp, ocol, val, oval) <= TOL[prec]


def test_grouped_mass_matrix():
    m = meshgen.config_mesh(2, n=11)
    compare_to_single(m, "fp64", 400, op="mass")


def test_grouped_flags_from_a_later_group():
    m = meshgen.config_mesh(3, n=6)
    conn = m.conn.copy()
    conn[m.n_elem - 5, 2] = m.n_node  # in the last group
    bad = meshgen.Mesh(4, conn, m.coords, m.coef)
    r = kb.build_lower_csr_grouped(*to_dev(bad), 4, 300, cap=box_nnz(4, 6, 6, 6), prec="fp64", check=False)
    assert r.flags & kb._lib.KB_F_INDEX
    # the element is left out, as by the single pass
    one = kb.build_lower_csr(*to_dev(bad), 4, prec="fp64", check=False)
    assert torch.equal(r.row_ptr, one.row_ptr) and torch.equal(r.col_idx, one.col_idx)


def test_grouped_capacity():
    m = meshgen.config_mesh(3, n=6)
    nnz = box_nnz(4, 6, 6, 6)
    ok = kb.build_lower_csr_grouped(*to_dev(m), 4, 200, cap=nnz, prec="fp64")
    assert ok.nnz == nnz
    short = kb.build_lower_csr_grouped(*to_dev(m), 4, 200, cap=nnz - 1, prec="fp64", check=False)
    assert short.flags & kb._lib.KB_F_CAPACITY


def test_grouped_empty_mesh():
    m = meshgen.Mesh(4, np.zeros((0, 4), np.int32), np.zeros((5, 3)), np.zeros(0))
    r = kb.build_lower_csr_grouped(*to_dev(m), 4, 10, cap=0, prec="fp64")
    assert r.nnz == 0 and r.row_ptr.cpu().tolist() == [0] * 6


def test_grouped_beyond_one_pass():
    n = 337
    m = meshgen.config_mesh(6)
    T = m.n_elem * 10
    nnz = box_nnz(4, n, n, n)
    say(f"[grouped-large] nel={m.n_elem} nn={m.n_node} pairs={T} (one pass indexes < 2^31) nnz={nnz}")
    assert T >= 2 ** 31
    dev = to_dev(m)
    with pytest.raises(kb.KBuildError):  # a single pass cannot index this many pairs
        kb.plan(4, m.n_elem, m.n_node, "fp32fb64")
    group = (m.n_elem + 1) // 2
    r = kb.build_lower_csr_grouped(*dev, 4, group, cap=nnz, prec="fp32fb64")
    del dev
    torch.cuda.empty_cache()
    say(f"  nnz={r.nnz}")
    rows, col = check_pattern(m, r, (n, n, n))
    check_row_sums(r, rows, col, "fp32fb64")
    del rows, col
    check_sampled_rows(m, r, "fp32fb64", n_sample=400)


def test_grouped_heavy_row_takes_the_heavy_path():
    """A star of 20,000 tets around one node whose id is the largest: its row gathers
    80,000 pairs, more than a sub-bucket's table holds, so each pass sums it on the
    heavy path, with residuals carried between the groups."""
    m = meshgen.fan_mesh(20000, True, seed=3)
    compare_to_single(m, "fp64", 6000)
    compare_to_single(m, "fp32fb64", 6000)


@pytest.mark.parametrize("prec", ["fp64", "fp32fb64"])
def test_grouped_heavy_diagonal_across_workgroups(prec):
    """A star of 300,000 tets in two groups: each pass's heavy row has a diagonal of
    150,000 pairs (plus the carried sum in the second), more than one workgroup sums
    alone, so its leaf is summed by several workgroups, with residuals."""
    m = meshgen.fan_mesh(300000, True, seed=5)
    say(f"[grouped-big-leaf] {prec}")
    compare_to_single(m, prec, 150000)


@pytest.mark.parametrize("prec", ["fp32fb64", "fp64"])
def test_streamed_groups_from_host_memory(prec):
    """Connectivity and coefficients in pinned host memory, streamed group by group into
    two device staging buffers while the previous group's pass runs: the result is the
    device-resident grouped build's bit for bit (the same passes in the same order), on
    two runs in a row, and agrees with the oracle."""
    m = meshgen.config_mesh(3, n=40)
    group = m.n_elem // 4 + 17  # four groups, the last one short
    say(f"[streamed] {prec} nel={m.n_elem} group={group}")
    dev = to_dev(m)
    one = kb.build_lower_csr(*dev, 4, prec=prec)
    ref = kb.build_lower_csr_grouped(*dev, 4, group, cap=one.nnz, prec=prec)
    conn_h = torch.from_numpy(m.conn).pin_memory()
    coef_h = torch.from_numpy(m.coef).pin_memory()
    sb = kb.StreamedGroupedBuilder(4, m.n_elem, m.n_node, group, one.nnz, prec=prec)
    assert sb.n_groups == 4
    for _ in range(2):
        sb.run(conn_h, dev[1], coef_h)
        r = sb.result()
        assert r.nnz == ref.nnz
        assert torch.equal(r.row_ptr, ref.row_ptr) and torch.equal(r.col_idx, ref.col_idx)
        assert torch.equal(r.vals, ref.vals)
    orp, ocol, oval, _ = oracle.build_mesh(m)
    rp, col, val = (t.cpu().numpy() for t in (r.row_ptr, r.col_idx, r.vals))
    np.testing.assert_array_equal(rp, orp)
    np.testing.assert_array_equal(col, ocol)
    assert scaled_error(orp, ocol, val.astype(np.float64), oval) <= TOL[prec]
    with pytest.raises(ValueError):  # device tensors are refused: the path reads host memory
        sb.run(dev[0], dev[1], dev[2])


@pytest.mark.parametrize("prec", ["fp64", "fp32fb64"])
@pytest.mark.parametrize("slots", [512, 4096])
def test_grouped_table_slots(slots, prec):
    """The pass-3 table size set by hand in a grouped build (the passes that also write
    residuals, whose FP64 variant keeps a column array of its own: its largest table at
    4096 slots): bit for bit the grouped build with the built-in table size.  With 512
    slots and 32-row sub-buckets the randomly numbered tets' last sub-buckets overflow to
    the heavy path."""
    m = meshgen.config_mesh(3, n=14)
    dev = to_dev(m)
    cap = box_nnz(4, 14, 14, 14)
    ref = kb.build_lower_csr_grouped(*dev, m.elem, 5000, cap=cap, prec=prec)
    got = kb.build_lower_csr_grouped(*dev, m.elem, 5000, cap=cap, prec=prec,
                                     tuning=kb.Tuning(sub_bits=5, table_slots=slots))
    say(f"[grouped-slots] slots={slots} {prec} nnz={got.nnz}")
    assert got.nnz == ref.nnz
    for x, y in zip(np_csr(got), np_csr(ref)):
        assert np.array_equal(x.view(np.uint8), y.view(np.uint8))
