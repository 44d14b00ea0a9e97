"""Assembly with several degrees of freedom per node on the GPU (through the C ABI)
against the FP64 oracle: random symmetric element matrices (2 and 3 DOFs, bricks and
tetrahedra, every precision mode, several tiles with a ragged tail, many buckets), exact
one-rounding sums in FP32, the Kronecker identity k ⊗ I -> K ⊗ I against the scalar
assembly (also on a 262,144-brick mesh with 3 DOFs), data errors and an empty mesh.
"""
from __future__ import annotations

import math

import numpy as np
import pytest
import torch

import meshgen
import oracle
import paper_1501_04784_amd as kb
from tests.gpu_common import say

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # collected on CPU only when -m gpu is asked for explicitly
    pytest.skip("no GPU", allow_module_level=True)

DEV = torch.device("cuda:0")


def mesh(elem, seed):
    """Several pass-1 tiles with a ragged tail: 504 bricks or 600 tetrahedra."""
    dims = (9, 8, 7) if elem == 8 else (5, 5, 4)
    return meshgen.box_mesh(elem, *dims, jitter=0.2, coef=(0.5, 2.0), permute_nodes=True, permute_elems=True,
                            seed=seed)


def values_for(m, dof, prec, seed):
    k = meshgen.element_matrices(m.n_elem, m.elem * dof, seed)
    return k.astype(np.float64 if prec == "fp64" else np.float32)


def gpu_assemble(m, dof, prec, klow, tuning=None, check=True, conn=None):
    conn = m.conn if conn is None else conn
    return kb.assemble_lower_csr(torch.from_numpy(np.ascontiguousarray(conn)).to(DEV), m.n_node,
                                 torch.from_numpy(klow).to(DEV), m.elem, prec=prec, tuning=tuning, check=check,
                                 dof=dof)


def host(r):
    return r.row_ptr.cpu().numpy(), r.col_idx.cpu().numpy(), r.vals.cpu().numpy()


def exact_sums_f32(elem, dof, conn, klow32):
    """Per entry, the exact sum of its float32 contributions (math.fsum; exact here,
    since the sums span fewer than 53 bits) rounded once to float32: independent of
    the oracle and of the GPU code (test-side triplets)."""
    nd = elem * dof
    p_idx = np.array([p for p in range(nd) for q in range(p + 1)])
    q_idx = np.array([q for p in range(nd) for q in range(p + 1)])
    g = dof * conn[:, :, None].astype(np.int64) + np.arange(dof)[None, None, :]
    g = g.reshape(conn.shape[0], nd)
    gp, gq = g[:, p_idx].ravel(), g[:, q_idx].ravel()
    key = np.maximum(gp, gq) * (1 << 32) + np.minimum(gp, gq)
    v = klow32.astype(np.float64).ravel()
    order = np.argsort(key, kind="stable")
    key, v = key[order], v[order]
    starts = np.flatnonzero(np.r_[True, key[1:] != key[:-1]])
    ends = np.r_[starts[1:], len(key)]
    return np.array([np.float32(math.fsum(v[s:e])) for s, e in zip(starts, ends)], np.float32)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp32fb64"])
@pytest.mark.parametrize("dof", [2, 3])
@pytest.mark.parametrize("elem", [8, 4])
def test_dof_parity(elem, dof, prec):
    m = mesh(elem, 10 + dof)
    klow = values_for(m, dof, prec, 20 + dof)
    say(f"[dof] elem={elem} dof={dof} {prec} nel={m.n_elem} nn={m.n_node}")
    rp, col, val = host(gpu_assemble(m, dof, prec, klow))
    k64 = klow.astype(np.float64)
    orp, ocol, oval, of = oracle.assemble_lower_csr_dof(elem, dof, m.conn, m.n_node, k64)
    assert of == 0
    np.testing.assert_array_equal(rp, orp)
    np.testing.assert_array_equal(col, ocol)
    # per-entry magnitude: the sum of |contributions|
    _, _, mag, _ = oracle.assemble_lower_csr_dof(elem, dof, m.conn, m.n_node, np.abs(k64))
    val = val.astype(np.float64)
    if prec == "fp64":
        # exact sum rounded once against a sequential FP64 sum: within a few ulps of mag
        assert np.all(np.abs(val - oval) <= 1e-14 * mag)
    else:
        # exact sum rounded once to float32: at most half an ulp of float32 from the exact sum
        assert np.all(np.abs(val - oval) <= 2.0 ** -24 * np.abs(oval) + 1e-14 * mag)


@pytest.mark.parametrize("dof", [2, 3])
@pytest.mark.parametrize("elem", [8, 4])
def test_dof_fp32_sums_are_exact_then_rounded_once(elem, dof):
    m = mesh(elem, 30 + dof)
    klow = values_for(m, dof, "fp32", 40 + dof)
    rp, col, val = host(gpu_assemble(m, dof, "fp32", klow))
    want = exact_sums_f32(elem, dof, m.conn, klow)
    assert val.dtype == np.float32 and len(val) == len(want)
    np.testing.assert_array_equal(val.view(np.uint32), want.view(np.uint32))


@pytest.mark.parametrize("dof", [2, 3])
def test_dof_heavy_rows_exact(dof):
    """A fan of 6000 tets around one node numbered last, with dof components per node:
    each of the centre's dof rows holds about 18,000 dof entries, more than a table (the
    heavy path).  The pattern against the oracle, and every entry the exact sum of its
    float32 contributions rounded once."""
    m = meshgen.fan_mesh(6000, True, seed=8)
    klow = values_for(m, dof, "fp32", 50 + dof)
    say(f"[dof-heavy] dof={dof} nel={m.n_elem} nn={m.n_node}")
    rp, col, val = host(gpu_assemble(m, dof, "fp32", klow))
    orp, ocol, _, of = oracle.assemble_lower_csr_dof(4, dof, m.conn, m.n_node, klow.astype(np.float64))
    assert of == 0
    np.testing.assert_array_equal(rp, orp)
    np.testing.assert_array_equal(col, ocol)
    want = exact_sums_f32(4, dof, m.conn, klow)
    np.testing.assert_array_equal(val.view(np.uint32), want.view(np.uint32))

@pytest.mark.parametrize("tuning", [kb.Tuning(bucket_bits=3, sub_bits=1), kb.Tuning(block=128),
                                    kb.Tuning(bucket_bits=8, sub_bits=8)])
@pytest.mark.parametrize("dof", [2, 3])
def test_dof_tunings_give_identical_results(dof, tuning):
    """Bucket sizes and tile size change the order of the exact sums only: bitwise equal."""
    m = mesh(8 if dof == 3 else 4, 50 + dof)
    klow = values_for(m, dof, "fp64", 60 + dof)
    a = host(gpu_assemble(m, dof, "fp64", klow))
    b = host(gpu_assemble(m, dof, "fp64", klow, tuning=tuning))
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)


def kron_values(k1, elem, dof):
    """Packed lower triangles of k ⊗ I_dof from packed scalar ones (torch, on k1's device)."""
    nd = elem * dof
    src = []
    for p in range(nd):
        for q in range(p + 1):
            a, c = divmod(p, dof)
            b, c2 = divmod(q, dof)
            src.append(a * (a + 1) // 2 + b if c == c2 else -1)  # a >= b since p >= q and c == c2
    src = torch.tensor(src, device=k1.device)
    out = k1[:, src.clamp(min=0)]
    return torch.where(src[None, :] >= 0, out, torch.zeros_like(out)).contiguous()


def expected_kron_csr(rp, col, val, dof):
    """The lower CSR of K ⊗ I_dof with its structural zeros, from a scalar lower CSR (torch)."""
    n = rp.numel() - 1
    row = torch.repeat_interleave(torch.arange(n, device=rp.device), rp[1:] - rp[:-1])
    c = torch.arange(dof, device=rp.device)
    R = dof * row[:, None, None] + c[None, :, None]  # [nnz, c, c']
    C = dof * col.long()[:, None, None] + c[None, None, :]
    keep = (row != col.long())[:, None, None] | (c[None, None, :] <= c[None, :, None])
    V = torch.where(c[None, :, None] == c[None, None, :], val[:, None, None], torch.zeros_like(val)[:, None, None])
    R, C, V = R.expand(-1, dof, dof)[keep], C.expand(-1, dof, dof)[keep], V.expand(-1, dof, dof)[keep]
    key = R * (dof * n) + C
    order = torch.argsort(key)
    R, C, V = R[order], C[order], V[order]
    rp2 = torch.zeros(dof * n + 1, dtype=torch.int64, device=rp.device)
    rp2[1:] = torch.cumsum(torch.bincount(R, minlength=dof * n), 0)
    return rp2, C, V


def check_kron(m, dof, prec="fp64"):
    conn = torch.from_numpy(m.conn).to(DEV)
    coords = torch.from_numpy(m.coords).to(DEV)
    coef = torch.from_numpy(m.coef).to(DEV)
    k1, _ = kb.integrate_lower(conn, coords, coef, m.elem, prec=prec)
    s = kb.assemble_lower_csr(conn, m.n_node, k1, m.elem, prec=prec)
    d = kb.assemble_lower_csr(conn, m.n_node, kron_values(k1, m.elem, dof), m.elem, prec=prec, dof=dof)
    rp2, C, V = expected_kron_csr(s.row_ptr.long(), s.col_idx, s.vals, dof)
    assert torch.equal(d.row_ptr.long(), rp2)
    assert torch.equal(d.col_idx.long(), C)
    # the structural zeros add nothing and leave the exponent range alone: bitwise equal
    assert torch.equal(d.vals, V)
    return d.nnz


@pytest.mark.parametrize("dof", [2, 3])
@pytest.mark.parametrize("elem", [8, 4])
def test_dof_kronecker_identity(elem, dof):
    check_kron(mesh(elem, 70 + dof), dof)


def test_dof_kronecker_identity_262k_bricks():
    """A 64^3 brick mesh with 3 DOFs (78.6M element pairs), checked whole by the identity."""
    m = meshgen.box_mesh(8, 64, 64, 64, jitter=0.2, coef=(1e-2, 1e2), permute_nodes=True, permute_elems=True,
                         seed=81)
    say(f"[dof-large] nel={m.n_elem} nn={m.n_node}")
    nnz = check_kron(m, 3, prec="fp32")
    say(f"  nnz={nnz}")


def test_dof_data_errors_match_the_oracle():
    elem, dof = 8, 3
    m = mesh(elem, 90)
    conn = m.conn.copy()
    conn[3, 2] = m.n_node       # out of range
    conn[7, 5] = -4             # negative
    conn[11, 1] = conn[11, 6]   # repeated node
    klow = values_for(m, dof, "fp64", 91)
    r = gpu_assemble(m, dof, "fp64", klow, check=False, conn=conn)
    rp, col, val = host(r)
    orp, ocol, oval, of = oracle.assemble_lower_csr_dof(elem, dof, conn, m.n_node, klow)
    assert of == kb._lib.KB_F_INDEX | kb._lib.KB_F_REPEAT
    assert r.flags & 0xF == of
    np.testing.assert_array_equal(rp, orp)
    np.testing.assert_array_equal(col, ocol)
    _, _, mag, _ = oracle.assemble_lower_csr_dof(elem, dof, conn, m.n_node, np.abs(klow))
    assert np.all(np.abs(val - oval) <= 1e-14 * mag)
    with pytest.raises(kb.KBuildError):
        gpu_assemble(m, dof, "fp64", klow, check=True, conn=conn)


@pytest.mark.parametrize("dof", [2, 3])
def test_dof_empty_mesh(dof):
    m = meshgen.Mesh(4, np.zeros((0, 4), np.int32), np.zeros((7, 3)), np.zeros(0))
    r = gpu_assemble(m, dof, "fp64", np.zeros((0, (4 * dof) * (4 * dof + 1) // 2)))
    assert r.nnz == 0
    assert r.row_ptr.cpu().tolist() == [0] * (dof * 7 + 1)
