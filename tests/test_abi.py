"""Host-side checks of the C ABI (no GPU needed): exports, planning, argument errors."""
from __future__ import annotations

import ctypes
import os
import re

import pytest

from paper_1501_04784_amd import _lib
from paper_1501_04784_amd._lib import KbBatch, KbMesh, KbTuning

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "kbuild.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\*?\s+\**(kb_\w+)\s*\(", src, flags=re.M)))


def test_library_exports_every_declared_function():
    names = declared_functions()
    assert set(names) == set(_lib.EXPORTS)
    L = _lib.lib()
    for n in names:
        assert hasattr(L, n), n


def test_header_constants_match_binding():
    src = open(HEADER).read()
    consts = dict(re.findall(r"#define\s+(KB_\w+)\s+\(?(-?\d+)u?\)?", src))
    for name in ("KB_HEX8", "KB_TET4", "KB_FP64", "KB_FP32", "KB_FP32_FB64", "KB_OK", "KB_EINVAL", "KB_ERANGE",
                 "KB_ENOSPC", "KB_EHIP", "KB_STATUS_WORDS", "KB_F_INDEX", "KB_F_REPEAT", "KB_F_INVERTED",
                 "KB_F_NONFINITE", "KB_F_CAPACITY", "KB_N_STAGES", "KB_OP_STIFFNESS", "KB_OP_MASS"):
        assert int(consts[name]) == getattr(_lib, name), name


def test_struct_layout():
    assert ctypes.sizeof(KbMesh) == 48
    assert KbMesh.conn.offset == 24 and KbMesh.coef.offset == 40
    assert ctypes.sizeof(KbTuning) == 32 and KbTuning.stage_events.offset == 16
    assert KbTuning.seg_pairs.offset == 24 and KbTuning.table_slots.offset == 28


def _plan(elem, nel, nn, prec=0, tuning=None):
    m = KbMesh(elem, 0, nel, nn, None, None, None)
    ws = ctypes.c_size_t(0)
    nt = ctypes.c_int64(0)
    tu = ctypes.byref(tuning) if tuning is not None else None
    rc = _lib.lib().kb_plan(ctypes.byref(m), prec, tu, ctypes.byref(ws), ctypes.byref(nt))
    return rc, ws.value, nt.value


def test_version_and_strings():
    L = _lib.lib()
    assert L.kb_version() == 4
    assert L.kb_status_string(0) == b"ok"
    assert L.kb_status_string(-3) == b"workspace too small"
    assert L.kb_status_string(16) == b"nnz exceeds capacity"
    assert L.kb_status_string(12345) == b"unknown status"


@pytest.mark.parametrize("elem,te", [(8, 36), (4, 10)])
@pytest.mark.parametrize("prec", [0, 1, 2])
def test_plan_sizes(elem, te, prec):
    rc, ws, nt = _plan(elem, 1000, 1331, prec)
    assert rc == 0 and nt == 1000 * te
    vb = 8 if prec == 0 else 4
    # at least: (16-bit row in bucket, col, value) and (packed key, value) pair lists,
    # per-node row offsets
    assert ws >= nt * (10 + 2 * vb) + 4 * 1331
    assert ws % 256 == 0


def test_plan_fp64_brick_tile_falls_back_with_many_buckets():
    """FP64 bricks stage 256 elements per pass-1 tile unless their bucket counters no
    longer fit beside them in LDS (beyond about 2000 buckets); then the 192 tile, also when
    256 is asked for.  The tile shows in the workspace (one histogram row per tile)."""
    def t(b):
        return KbTuning(b, 0, 0.0, 0, None)
    few = [_plan(8, 10000, 60_000_000, 0, tuning=t(b)) for b in (0, 256, 192)]  # 1831 buckets
    assert all(r[0] == 0 for r in few) and few[0][1] == few[1][1] != few[2][1]
    many = [_plan(8, 10000, 80_000_000, 0, tuning=t(b)) for b in (0, 256, 192)]  # 4883 buckets
    assert all(r[0] == 0 for r in many) and many[0][1] == many[1][1] == many[2][1]


def test_plan_empty_mesh():
    rc, ws, nt = _plan(4, 0, 0)
    assert rc == 0 and nt == 0


def test_plan_errors():
    L = _lib.lib()
    assert L.kb_plan(None, 0, None, None, None) == _lib.KB_EINVAL
    assert _plan(5, 10, 10)[0] == _lib.KB_EINVAL
    assert _plan(8, 10, 10, prec=3)[0] == _lib.KB_EINVAL
    assert _plan(8, -1, 10)[0] == _lib.KB_EINVAL
    assert _plan(8, 10, -1)[0] == _lib.KB_EINVAL
    assert _plan(8, 2**31 // 36 + 1, 10)[0] == _lib.KB_ERANGE
    assert _plan(4, 10, 2**31)[0] == _lib.KB_ERANGE
    assert _plan(4, 2**31 // 10, 10)[0] == 0
    assert _plan(8, 10, 10, tuning=KbTuning(100, 0, 0.0, 0, None))[0] == _lib.KB_EINVAL  # block not multiple of 64
    assert _plan(8, 10, 10, tuning=KbTuning(0, 31, 0.0, 0, None))[0] == _lib.KB_EINVAL  # bucket bits
    assert _plan(8, 10, 10, tuning=KbTuning(0, 17, 0.0, 8, None))[0] == _lib.KB_EINVAL  # rows in bucket > 2^16
    assert _plan(8, 10, 10, tuning=KbTuning(0, 0, 0.5, 0, None))[0] == _lib.KB_EINVAL  # tau <= 1
    assert _plan(8, 10, 10, tuning=KbTuning(0, 0, 0.0, 9, None))[0] == _lib.KB_EINVAL  # sub-bucket bits > 8
    assert _plan(8, 10, 10, tuning=KbTuning(0, 3, 0.0, 5, None))[0] == _lib.KB_EINVAL  # sub > bucket
    assert _plan(8, 10, 10, tuning=KbTuning(0, 20, 0.0, 2, None))[0] == _lib.KB_EINVAL  # > 1024 sub-buckets
    assert _plan(8, 10, 10, tuning=KbTuning(512, 10, 8.0, 4, None))[0] == 0
    assert _plan(8, 10, 10, tuning=KbTuning(0, 0, 0.0, 0, None, 2048, 0))[0] == _lib.KB_EINVAL  # segment length
    for slots in (1, 256, 768, 8192, -1024):  # table slots: a power of two in [512, 4096]
        assert _plan(8, 10, 10, tuning=KbTuning(0, 0, 0.0, 0, None, 0, slots))[0] == _lib.KB_EINVAL
    for slots in (512, 1024, 2048, 4096):
        assert _plan(4, 1000, 300, tuning=KbTuning(0, 0, 0.0, 5, None, 0, slots))[0] == 0
    assert _plan(8, 10, 10, tuning=KbTuning(0, 0, 0.0, 0, None, 8192, 0))[0] == 0
    assert _plan(4, 10, 10, tuning=KbTuning(0, 0, 0.0, 0, None, 4096, 0))[0] == 0


def test_build_argument_errors_return_before_any_launch():
    """Null pointers and short workspaces are rejected on the host (no device touched)."""
    L = _lib.lib()
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: every call below fails validation first
    m = KbMesh(8, 0, 10, 20, 0x1000, 0x1000, 0x1000)
    rc, ws, nt = _plan(8, 10, 20)
    args = dict(ws=fake, ws_bytes=ws, row_ptr=fake, col=fake, vals=fake, cap=nt, nnz=fake, status=fake)

    def call(**kw):
        a = {**args, **kw}
        return L.kb_build_lower_csr(ctypes.byref(m), 0, None, a["ws"], a["ws_bytes"], a["row_ptr"], a["col"],
                                    a["vals"], a["cap"], a["nnz"], a["status"], None)

    assert call(ws_bytes=ws - 1) == _lib.KB_ENOSPC
    assert call(row_ptr=None) == _lib.KB_EINVAL
    assert call(nnz=None) == _lib.KB_EINVAL
    assert call(status=None) == _lib.KB_EINVAL
    assert call(cap=-1) == _lib.KB_EINVAL
    assert call(col=None) == _lib.KB_EINVAL
    assert call(ws=None) == _lib.KB_EINVAL
    m.conn = None
    assert call() == _lib.KB_EINVAL
    m.conn = 0x1000
    m.coords = None
    assert call() == _lib.KB_EINVAL
    # assembly-only path does not need coordinates, but needs values
    assert L.kb_assemble_lower_csr(ctypes.byref(m), 0, None, None, fake, ws, fake, fake, fake, nt, fake, fake,
                                   None) == _lib.KB_EINVAL
    assert L.kb_integrate_lower(ctypes.byref(m), 0, None, fake, None, None) == _lib.KB_EINVAL


def test_batch_struct_layout():
    assert ctypes.sizeof(KbBatch) == 64
    assert KbBatch.elem_off.offset == 24 and KbBatch.coef.offset == 56


def test_plan_batched_adds_packing_space():
    L = _lib.lib()
    b = KbBatch(8, 3, 1000, 1331, None, None, None, None, None)
    ws, nt = ctypes.c_size_t(0), ctypes.c_int64(0)
    assert L.kb_plan_batched(ctypes.byref(b), 0, None, ctypes.byref(ws), ctypes.byref(nt)) == 0
    rc, ws1, nt1 = _plan(8, 1000, 1331)
    assert nt.value == nt1 and ws.value >= ws1 + 4 * 8 * 1000 + 4 * 1332
    b.n_mesh = -1
    assert L.kb_plan_batched(ctypes.byref(b), 0, None, ctypes.byref(ws), ctypes.byref(nt)) == _lib.KB_EINVAL
    assert L.kb_plan_batched(None, 0, None, None, None) == _lib.KB_EINVAL


def test_build_batched_argument_errors():
    L = _lib.lib()
    fake = 0x1000
    b = KbBatch(8, 2, 10, 20, fake, fake, fake, fake, fake)
    ws, nt = ctypes.c_size_t(0), ctypes.c_int64(0)
    assert L.kb_plan_batched(ctypes.byref(b), 0, None, ctypes.byref(ws), ctypes.byref(nt)) == 0
    f = ctypes.c_void_p(fake)

    def call(**kw):
        a = dict(ws=f, wsb=ws.value, rp=f, col=f, val=f, cap=nt.value, off=f, st=f)
        a.update(kw)
        return L.kb_build_lower_csr_batched(ctypes.byref(b), 0, None, a["ws"], a["wsb"], a["rp"], a["col"], a["val"],
                                            a["cap"], a["off"], a["st"], None)

    assert call(wsb=ws.value - 1) == _lib.KB_ENOSPC
    assert call(rp=None) == _lib.KB_EINVAL
    assert call(off=None) == _lib.KB_EINVAL
    assert call(st=None) == _lib.KB_EINVAL
    assert call(ws=None) == _lib.KB_EINVAL
    b.elem_off = None
    assert call() == _lib.KB_EINVAL
    b.elem_off = fake
    b.coords = None
    assert call() == _lib.KB_EINVAL


def test_plan_adjoint_and_argument_errors():
    L = _lib.lib()
    m = KbMesh(8, 0, 100, 200, 0x1000, 0x1000, 0x1000)
    ws = ctypes.c_size_t(0)
    assert L.kb_plan_adjoint(ctypes.byref(m), ctypes.byref(ws)) == 0
    assert ws.value >= 8 * 3 * 8 * 100 + 16 * 3 * 200
    assert L.kb_plan_adjoint(None, ctypes.byref(ws)) == _lib.KB_EINVAL
    f = ctypes.c_void_p(0x1000)

    def call(**kw):
        a = dict(rp=f, col=f, w=f, nnz=10, ws=f, wsb=ws.value, gc=f, gx=f, st=f)
        a.update(kw)
        return L.kb_adjoint_lower(ctypes.byref(m), a["rp"], a["col"], a["w"], a["nnz"], a["ws"], a["wsb"], a["gc"],
                                  a["gx"], a["st"], None)

    assert call(wsb=ws.value - 1) == _lib.KB_ENOSPC
    for k in ("rp", "col", "w", "ws", "gc", "gx", "st"):
        assert call(**{k: None}) == _lib.KB_EINVAL, k
    assert call(nnz=-1) == _lib.KB_EINVAL
    assert call(nnz=1 << 31) == _lib.KB_ERANGE
    bad = KbMesh(5, 0, 100, 200, 0x1000, 0x1000, 0x1000)
    assert L.kb_plan_adjoint(ctypes.byref(bad), ctypes.byref(ws)) == _lib.KB_EINVAL


def test_operator_field():
    L = _lib.lib()
    ws0, ws1 = ctypes.c_size_t(0), ctypes.c_size_t(0)
    m = KbMesh(4, 0, 1000, 500, None, None, None)
    assert L.kb_plan(ctypes.byref(m), 1, None, ctypes.byref(ws0), None) == 0
    m.op = 1  # mass: integrated in pass 1 like the stiffness matrix, same workspace
    assert L.kb_plan(ctypes.byref(m), 1, None, ctypes.byref(ws1), None) == 0
    assert ws1.value == ws0.value
    m.op = 2
    assert L.kb_plan(ctypes.byref(m), 1, None, ctypes.byref(ws1), None) == _lib.KB_EINVAL
    m.op = 1  # the adjoint is for the stiffness matrix only
    assert L.kb_plan_adjoint(ctypes.byref(m), ctypes.byref(ws1)) == _lib.KB_EINVAL


def _plan_dof(elem, nel, nn, dof, prec=0):
    m = KbMesh(elem, 0, nel, nn, None, None, None)
    ws, nt = ctypes.c_size_t(0), ctypes.c_int64(0)
    rc = _lib.lib().kb_plan_dof(ctypes.byref(m), dof, prec, None, ctypes.byref(ws), ctypes.byref(nt))
    return rc, ws.value, nt.value


@pytest.mark.parametrize("elem", [8, 4])
def test_plan_dof(elem):
    # dof 1 is the scalar plan
    assert _plan_dof(elem, 1000, 900, 1) == _plan(elem, 1000, 900)
    for dof in (2, 3):
        nd = elem * dof
        rc, ws, nt = _plan_dof(elem, 1000, 900, dof)
        assert rc == 0 and nt == 1000 * nd * (nd + 1) // 2
        # at least: expanded connectivity, pass-1 and pass-2 streams, dof * n_node row offsets
        assert ws >= 4 * nd * 1000 + (2 + 4 + 8 + 4 + 8) * nt + 4 * dof * 900
    for dof in (0, 4, -1):
        assert _plan_dof(elem, 10, 10, dof)[0] == _lib.KB_EINVAL
    # dof * n_node must stay below 2^31
    assert _plan_dof(elem, 10, (1 << 31) // 3, 3)[0] == _lib.KB_ERANGE
    assert _plan_dof(elem, 10, (1 << 25) - 1, 2)[0] == 0  # 2^26 rows
    # triplets of int32 indexing
    nd = elem * 3
    assert _plan_dof(elem, (1 << 31) // (nd * (nd + 1) // 2) + 1, 100, 3)[0] == _lib.KB_ERANGE


def test_assemble_dof_argument_errors():
    L = _lib.lib()
    m = KbMesh(8, 0, 100, 200, 0x1000, None, None)
    ws, nt = ctypes.c_size_t(0), ctypes.c_int64(0)
    assert L.kb_plan_dof(ctypes.byref(m), 3, 0, None, ctypes.byref(ws), ctypes.byref(nt)) == 0
    f = ctypes.c_void_p(0x1000)

    def call(**kw):
        a = dict(dof=3, kl=f, ws=f, wsb=ws.value, rp=f, col=f, val=f, cap=nt.value, nnz=f, st=f)
        a.update(kw)
        return L.kb_assemble_lower_csr_dof(ctypes.byref(m), a["dof"], 0, None, a["kl"], a["ws"], a["wsb"], a["rp"],
                                           a["col"], a["val"], a["cap"], a["nnz"], a["st"], None)

    assert call(wsb=ws.value - 1) == _lib.KB_ENOSPC
    assert call(dof=4) == _lib.KB_EINVAL
    assert call(cap=-1) == _lib.KB_EINVAL
    for k in ("kl", "ws", "rp", "nnz", "st"):
        assert call(**{k: None}) == _lib.KB_EINVAL, k
    for k in ("col", "val"):  # needed only when cap > 0
        assert call(**{k: None}) == _lib.KB_EINVAL, k
    m.conn = None
    assert call() == _lib.KB_EINVAL


def _plan_grouped(elem, nel, nn, group, cap, prec=1):
    m = KbMesh(elem, 0, nel, nn, None, None, None)
    ws = ctypes.c_size_t(0)
    rc = _lib.lib().kb_plan_grouped(ctypes.byref(m), prec, None, group, cap, ctypes.byref(ws))
    return rc, ws.value


def test_plan_grouped():
    # one group is the single pass
    rc, ws1 = _plan_grouped(4, 1000, 300, 5000, 2000)
    assert rc == 0 and ws1 >= _plan(4, 1000, 300, 1)[1]
    # several groups carry the sums: workspace grows with the capacity
    rc, wa = _plan_grouped(4, 1000, 300, 100, 2000)
    rc2, wb = _plan_grouped(4, 1000, 300, 100, 4000)
    assert rc == 0 and rc2 == 0 and wb > wa
    assert _plan_grouped(4, 1000, 300, 0, 10)[0] == _lib.KB_EINVAL
    assert _plan_grouped(4, 1000, 300, 10, -1)[0] == _lib.KB_EINVAL
    # a pass's pairs: group * 10 + 2 * cap must stay below 2^31
    assert _plan_grouped(4, 10 ** 9, 10 ** 6, 10 ** 8, 6 * 10 ** 8)[0] == _lib.KB_ERANGE


def test_plan_grouped_beyond_one_pass():
    """The Kuhn box 6 x 337^3: too many pairs for one pass, two groups fit."""
    nel, nn, nnz = 6 * 337 ** 3, 338 ** 3, 307_546_875
    assert _plan(4, nel, nn, 1)[0] == _lib.KB_ERANGE
    rc, ws = _plan_grouped(4, nel, nn, (nel + 1) // 2, nnz)
    assert rc == 0
    assert ws < 80 * 2 ** 30  # well inside one GPU's memory


def test_grouped_argument_errors():
    L = _lib.lib()
    m = KbMesh(4, 0, 1000, 300, 0x1000, 0x1000, 0x1000)
    ws = ctypes.c_size_t(0)
    assert L.kb_plan_grouped(ctypes.byref(m), 1, None, 100, 5000, ctypes.byref(ws)) == 0
    f = ctypes.c_void_p(0x1000)

    def call(**kw):
        a = dict(g=100, ws=f, wsb=ws.value, rp=f, col=f, val=f, cap=5000, nnz=f, st=f)
        a.update(kw)
        return L.kb_build_lower_csr_grouped(ctypes.byref(m), 1, None, a["g"], a["ws"], a["wsb"], a["rp"], a["col"],
                                            a["val"], a["cap"], a["nnz"], a["st"], None)

    assert call(wsb=ws.value - 1) == _lib.KB_ENOSPC
    assert call(g=0) == _lib.KB_EINVAL
    for k in ("ws", "rp", "col", "val", "nnz", "st"):
        assert call(**{k: None}) == _lib.KB_EINVAL, k


def test_noalloc_host_errors_before_any_device_call():
    """kb_build_lower_csr_noalloc checks its arguments and the mesh's workspace figure
    against the fixed scratch size on the host, before it looks up the scratch array."""
    L = _lib.lib()
    fake = ctypes.c_void_p(0x1000)  # never dereferenced
    src = open(HEADER).read()
    scratch = int(eval(re.search(r"#define\s+KB_SCRATCH_BYTES\s+\((\d+)u\s*<<\s*(\d+)\)", src).expand(r"\1 << \2")))
    assert scratch == _lib.KB_SCRATCH_BYTES

    def call(m, prec=1, row_ptr=fake, cap=10):
        return L.kb_build_lower_csr_noalloc(ctypes.byref(m), prec, None, row_ptr, fake, fake, cap, fake, fake, None)

    # the largest tet mesh whose workspace fits, and one beyond (plan figures only)
    ok = KbMesh(4, 0, 200_000, 40_000, 0x1000, 0x1000, 0x1000)
    assert _plan(4, 200_000, 40_000, 1)[1] <= scratch
    big = KbMesh(4, 0, 2_000_000, 400_000, 0x1000, 0x1000, 0x1000)
    assert _plan(4, 2_000_000, 400_000, 1)[1] > scratch
    assert call(big) == _lib.KB_ENOSPC
    assert call(KbMesh(5, 0, 10, 10, 0x1000, 0x1000, 0x1000)) == _lib.KB_EINVAL
    assert call(ok, prec=7) == _lib.KB_EINVAL
    assert call(ok, row_ptr=None) == _lib.KB_EINVAL
    assert call(ok, cap=-1) == _lib.KB_EINVAL
    ok.coords = None
    assert call(ok) == _lib.KB_EINVAL


@pytest.mark.parametrize("elem", [4, 8])
@pytest.mark.parametrize("prec", [0, 2])
def test_plan_widens_buckets_for_very_many_rows(elem, prec):
    """With the default tuning, the plan widens the row buckets (and narrows the tile) so
    that pass 1's bucket counters fit in LDS: up to 2^27 rows; 2^28 rows are refused (the
    sub-bucket key has no room left for the row beside a 28-bit column)."""
    for nn in (80_000_000, 2**27):
        nel = min(nn * (6 if elem == 4 else 1), 2**31 // (10 if elem == 4 else 36) - 1)
        rc, ws, nt = _plan(elem, nel, nn, prec)
        assert rc == 0, nn
    assert _plan(elem, 1000, 2**28, prec)[0] == _lib.KB_EINVAL
