"""Consistent mass matrix on the GPU (same construction, another integrand: Section 5)
against the FP64 oracle's, which is pinned separately (closed forms, total mass, a second
route).  Pattern exact; values to the same diagonal-scaled tolerances as the stiffness
matrix (the mass matrix is positive definite, so the scale is always positive)."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import meshgen
import oracle
import paper_1501_04784_amd as kb
from tests.gpu_common import TOL, elem_scaled_error, say, to_dev
from tests.helpers import scaled_error

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # collected on CPU only when -m gpu is asked for explicitly
    pytest.skip("no GPU", allow_module_level=True)

MESHES = {
    "hex_perm": meshgen.box_mesh(8, 9, 7, 6, jitter=0.25, coef=(1e-2, 1e2), permute_nodes=True, permute_elems=True,
                                 seed=41),
    "tet_perm": meshgen.box_mesh(4, 8, 6, 7, jitter=0.2, coef=(1e-3, 1e3), permute_nodes=True, permute_elems=True,
                                 seed=42),
    "c3_tet20": meshgen.config_mesh(3, n=20),
}


@pytest.mark.parametrize("prec", ["fp64", "fp32fb64", "fp32"])
@pytest.mark.parametrize("name", sorted(MESHES))
def test_mass_build_parity(name, prec):
    m = MESHES[name]
    say(f"[mass] {name} {prec} nel={m.n_elem}")
    conn, coords, coef = to_dev(m)
    r = kb.build_lower_csr(conn, coords, coef, m.elem, prec=prec, op="mass")
    orp, ocol, oval, f = oracle.build_mass_mesh(m)
    assert f == 0
    np.testing.assert_array_equal(r.row_ptr.cpu().numpy(), orp)
    np.testing.assert_array_equal(r.col_idx.cpu().numpy(), ocol)
    err = scaled_error(orp, ocol, r.vals.cpu().numpy().astype(np.float64), oval)
    say(f"  scaled error {err:.3e}")
    assert err <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name", ["hex_perm", "tet_perm"])
def test_mass_integrate_parity(name, prec):
    m = MESHES[name]
    conn, coords, coef = to_dev(m)
    k, _ = kb.integrate_lower(conn, coords, coef, m.elem, prec=prec, op="mass")
    kref, f = oracle.integrate_mass_lower(m.elem, m.conn, m.coords, m.coef)
    assert f == 0
    assert elem_scaled_error(k.cpu().numpy().astype(np.float64), kref, m.elem) <= TOL[prec]


def test_mass_and_stiffness_share_the_pattern():
    m = MESHES["tet_perm"]
    conn, coords, coef = to_dev(m)
    a = kb.build_lower_csr(conn, coords, coef, m.elem, prec="fp64", op="mass")
    b = kb.build_lower_csr(conn, coords, coef, m.elem, prec="fp64")
    assert torch.equal(a.row_ptr, b.row_ptr) and torch.equal(a.col_idx, b.col_idx)
