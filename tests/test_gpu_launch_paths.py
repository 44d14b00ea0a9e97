"""Every launch path of the build compared with the FP64 oracle entry by entry.

* The whole 20.25M-tet workload (Kuhn 6 x 150^3, random node and element numbering) in
  the benchmark's own launch configuration: each persistent pass-1 workgroup walks
  tens of tiles through its next-tile prefetch, and the sub-bucket partition takes the
  8192-pair segments with 512 sub-buckets per bucket.  All 27,270,901 entries are
  compared with the oracle's (pattern bit for bit, values within the precision's
  diagonal-scaled tolerance), for FP32 with FP64 fallback and for FP64.
* The same paths at sizes the oracle finishes in seconds: the half tiles (512 / 384
  elements) on a mesh with several tiles per workgroup, and a tuning that forces the
  long segments and 512 sub-buckets per bucket on a small mesh.
* Pass-3 hash tables sized by hand, down to one slot per expected entry, and the tuning
  search's choice for one mesh.
"""
from __future__ import annotations

import time

import numpy as np
import pytest
import torch

import meshgen
import oracle
import paper_1501_04784_amd as kb
from tests.gpu_common import TOL, np_csr, say, to_dev
from tests.helpers import box_nnz, scaled_error

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # collected on CPU only when -m gpu is asked for explicitly
    pytest.skip("no GPU", allow_module_level=True)

_FULL = {}


def full_c3():
    """(mesh, oracle CSR) of the whole 20.25M-tet workload, computed once per session."""
    if not _FULL:
        t = time.perf_counter()
        m = meshgen.config_mesh(3)
        say(f"  workload generated in {time.perf_counter() - t:.1f} s; running the oracle on all "
            f"{m.n_elem:,} elements")
        t = time.perf_counter()
        orp, ocol, oval, oflags = oracle.build_mesh(m)
        say(f"  oracle done in {time.perf_counter() - t:.1f} s, nnz {len(ocol):,}")
        assert oflags == 0
        _FULL.update(mesh=m, ref=(orp, ocol, oval))
    return _FULL["mesh"], _FULL["ref"]


def compare(m, r, ref, prec):
    rp, col, val = np_csr(r)
    orp, ocol, oval = ref
    np.testing.assert_array_equal(rp, orp)
    np.testing.assert_array_equal(col, ocol)
    err = scaled_error(orp, ocol, val, oval)
    say(f"  nnz={len(col):,} all entries compared, scaled error {err:.3e}, fallback={r.n_fallback}")
    assert err <= TOL[prec]
    return err


@pytest.mark.parametrize("prec", ["fp32fb64", "fp64"])
def test_c3_full_every_entry(prec):
    say(f"[c3-full] tet 6x150^3 {prec}: every entry against the oracle")
    m, ref = full_c3()
    r = kb.build_lower_csr(*to_dev(m), m.elem, prec=prec)
    assert r.nnz == box_nnz(4, 150, 150, 150) == 27270901
    compare(m, r, ref, prec)


@pytest.mark.parametrize("prec,block", [("fp32fb64", 512), ("fp64", 384), ("fp32fb64", 1024), ("fp64", 768)])
def test_tet_tiles_several_per_workgroup(prec, block):
    """1.3M randomly numbered tets: every tet pass-1 tile walks several tiles per
    persistent workgroup (the half tiles: about five per workgroup)."""
    m = meshgen.config_mesh(3, n=60)
    say(f"[tet-tiles] {prec} block={block} nel={m.n_elem:,}")
    r = kb.build_lower_csr(*to_dev(m), m.elem, prec=prec, tuning=kb.Tuning(block=block))
    ref = oracle.build_mesh(m)
    assert ref[3] == 0
    compare(m, r, ref[:3], prec)


@pytest.mark.parametrize("prec", ["fp32fb64", "fp64"])
def test_long_segments_many_sub_buckets(prec):
    """16384-row buckets of 32-row sub-buckets (512 per bucket) on a small tet mesh: the
    8192-pair segments of the sub-bucket histogram and scatter, as on the full workload."""
    m = meshgen.config_mesh(3, n=30)
    say(f"[long-seg] {prec} nel={m.n_elem:,}")
    r = kb.build_lower_csr(*to_dev(m), m.elem, prec=prec, tuning=kb.Tuning(bucket_bits=14, sub_bits=5))
    ref = oracle.build_mesh(m)
    compare(m, r, ref[:3], prec)


@pytest.mark.parametrize("cid,n,sub_bits,slots", [(3, 30, 5, 512), (3, 30, 4, 4096), (7, 40, 5, 1024), (7, 40, 6, 512)])
def test_table_slots(cid, n, sub_bits, slots):
    """The pass-3 table size set by hand, with wider sub-buckets: randomly numbered tets
    with half-size tables (the last rows' sub-buckets, which hold about twice the
    average entries, overflow to the heavy path), a table of 4096 slots, and naturally
    numbered bricks at two and one slots per expected entry.  Every entry against the
    oracle, and bit for bit the matrix of the default launch."""
    m = meshgen.config_mesh(cid, n=n)
    prec = "fp32fb64" if cid == 3 else "fp64"
    say(f"[table-slots] cid={cid} n={n} sub_bits={sub_bits} slots={slots} nel={m.n_elem:,} {prec}")
    dev = to_dev(m)
    r = kb.build_lower_csr(*dev, m.elem, prec=prec, tuning=kb.Tuning(sub_bits=sub_bits, table_slots=slots))
    d = kb.build_lower_csr(*dev, m.elem, prec=prec)
    for x, y in zip(np_csr(r), np_csr(d)):
        assert np.array_equal(x.view(np.uint8), y.view(np.uint8))
    ref = oracle.build_mesh(m)
    compare(m, r, ref[:3], prec)


def test_tune_build_valid_cached_and_bit_equal(tmp_path):
    """The tuning search on one naturally numbered brick mesh: the choice is valid for
    the shape, stored in the JSON cache and read back from it, never slower than the
    built-in choice in the search's own timing, and builds the same matrix bit for bit."""
    m = meshgen.config_mesh(7, n=24)
    dev = to_dev(m)
    cache = str(tmp_path / "tuning.json")
    t, entry = kb.tune_build(*dev, m.elem, "fp64", cache_path=cache)
    say(f"[tune-build] chose {t} in {entry['ms']:.3f} ms (built-in {entry['default_ms']:.3f} ms, "
        f"{entry['candidates_timed']} candidates timed)")
    assert entry["source"] == "search" and entry["candidates_timed"] >= 4
    assert entry["ms"] <= entry["default_ms"]
    kb.plan(m.elem, m.n_elem, m.n_node, "fp64", t)  # valid
    t2, entry2 = kb.tune_build(*dev, m.elem, "fp64", cache_path=cache)
    assert entry2["source"] == "cache" and t2 == t
    r = kb.build_lower_csr(*dev, m.elem, prec="fp64", tuning=t)
    d = kb.build_lower_csr(*dev, m.elem, prec="fp64")
    for x, y in zip(np_csr(r), np_csr(d)):
        assert np.array_equal(x.view(np.uint8), y.view(np.uint8))
    ref = oracle.build_mesh(m)
    compare(m, r, ref[:3], "fp64")
