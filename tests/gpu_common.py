"""Helpers for the GPU tests: run the HIP path through the C ABI, compare with the oracle."""
from __future__ import annotations

import sys

import numpy as np
import torch

import paper_1501_04784_amd as kb

TOL = {"fp64": 1e-12, "fp32fb64": 5e-6, "fp32": 2e-5}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(mesh):
    d = torch.device("cuda:0")
    return (torch.from_numpy(mesh.conn).to(d), torch.from_numpy(mesh.coords).to(d), torch.from_numpy(mesh.coef).to(d))


def gpu_build(mesh, prec, tuning=None, allow_flags=0, check=True, cap=None):
    conn, coords, coef = to_dev(mesh)
    r = kb.build_lower_csr(conn, coords, coef, mesh.elem, prec=prec, tuning=tuning, check=check,
                           allow_flags=allow_flags, cap=cap)
    return r


def np_csr(r):
    return (r.row_ptr.cpu().numpy(), r.col_idx.cpu().numpy(), r.vals.cpu().numpy().astype(np.float64))


def elem_scaled_error(k_gpu, k_ref, nen):
    """Per element max |dk_ab| / sqrt(k_aa k_bb) (reference diagonal)."""
    diag_idx = [a * (a + 1) // 2 + a for a in range(nen)]
    d = np.abs(k_ref[:, diag_idx])
    a_idx = np.array([a for a in range(nen) for b in range(a + 1)])
    b_idx = np.array([b for a in range(nen) for b in range(a + 1)])
    scale = np.sqrt(d[:, a_idx] * d[:, b_idx])
    scale = np.where(scale > 0, scale, 1.0)
    return float(np.max(np.abs(k_gpu - k_ref) / scale)) if k_ref.size else 0.0
