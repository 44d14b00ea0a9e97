"""Seeded synthetic mesh generators: the inputs shared by the oracle and the HIP path.

This module only builds input arrays (connectivity ``conn``, nodal coordinates
``coords`` and the per-element coefficient ``coef``, i.e. the paper's E, C and
MP arrays of Section 3).  It contains none of the method's arithmetic: no
shape functions, Jacobians, quadrature or assembly.  Tet orientation is fixed
combinatorially (by the parity of the axis permutation of each Kuhn simplex),
never from coordinates.

Recipe (all draws from numpy ``default_rng`` streams spawned from
``SeedSequence(seed)``; stream order: jitter, node permutation, element
permutation, coefficient, loss weights, spare):

* Domain: a box of ``nx*ny*nz`` cubic cells of edge ``h`` starting at the
  origin; node (i, j, k) has id ``i + (nx+1)*(j + (ny+1)*k)`` and position
  ``(i, j, k)*h`` before jitter; cell (i, j, k) has id ``i + nx*(j + ny*k)``.
* Jitter: interior nodes only, each coordinate i.i.d. U[-jitter*h, +jitter*h];
  boundary nodes stay on the box faces so the domain volume is exact.
* hex8: local corner order (0,0,0) (1,0,0) (1,1,0) (0,1,0) (0,0,1) (1,0,1)
  (1,1,1) (0,1,1) (cell offsets), i.e. counter-clockwise bottom face then top.
* tet4: each cell split into the six Kuhn simplices, one per axis permutation
  p (lexicographic order): v0 = cell corner, v1 = v0 + e_p0, v2 = v1 + e_p1,
  v3 = v0 + (1,1,1); for odd p, v2 and v3 are swapped so that every tet is
  positively oriented in the undistorted grid.
* Optional uniformly random node relabelling and element reordering.
* Coefficient: constant, or log-uniform ``exp(U[ln lo, ln hi])``.

A fan (``fan_mesh``) is n tets around one shared node: tet t is (centre, 1+3t, 2+3t,
3+3t) with its three corners at ``s * R (I + E)`` rows, E i.i.d. U[-0.2, 0.2] (so
``||E|| < 1`` and I + E keeps the positive orientation of the unit corner tet), s
U[0.5, 2] and R a proper rotation from a normalised Gaussian quaternion; coefficient
``exp(U[-2, 2])``.  With ``center_last`` the centre takes the largest id (the others
shift down by one), so that its row holds every element's pairs.
"""
from __future__ import annotations

import hashlib
import itertools
from dataclasses import dataclass, field

import numpy as np

HEX_CORNERS = np.array(
    [(0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0), (0, 0, 1), (1, 0, 1), (1, 1, 1), (0, 1, 1)],
    dtype=np.int64,
)
KUHN_PERMS = list(itertools.permutations(range(3)))  # lexicographic


def _perm_is_odd(p) -> bool:
    inv = sum(1 for a in range(3) for b in range(a + 1, 3) if p[a] > p[b])
    return inv % 2 == 1


@dataclass
class Mesh:
    """One mesh: ``elem`` is 8 (hex8) or 4 (tet4)."""

    elem: int
    conn: np.ndarray  # int32 [n_elem, nen], 0-based node ids
    coords: np.ndarray  # float64 [n_node, 3]
    coef: np.ndarray  # float64 [n_elem]
    meta: dict = field(default_factory=dict)

    @property
    def n_elem(self) -> int:
        return int(self.conn.shape[0])

    @property
    def n_node(self) -> int:
        return int(self.coords.shape[0])

    @property
    def nen(self) -> int:
        return int(self.conn.shape[1])

    def sha256(self) -> str:
        h = hashlib.sha256()
        for a in (self.conn, self.coords, self.coef):
            h.update(np.ascontiguousarray(a).tobytes())
        return h.hexdigest()


def streams(seed: int, k: int = 6):
    return [np.random.default_rng(s) for s in np.random.SeedSequence(seed).spawn(k)]


def _grid_nodes(nx, ny, nz, h, jitter, rng):
    i, j, k = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), np.arange(nz + 1), indexing="ij")
    # node id = i + (nx+1)*(j + (ny+1)*k): flatten with i fastest
    ijk = np.stack([i.ravel(order="F"), j.ravel(order="F"), k.ravel(order="F")], axis=1)
    coords = ijk.astype(np.float64) * h
    if jitter > 0:
        interior = (
            (ijk[:, 0] > 0) & (ijk[:, 0] < nx) & (ijk[:, 1] > 0) & (ijk[:, 1] < ny)
            & (ijk[:, 2] > 0) & (ijk[:, 2] < nz)
        )
        d = rng.uniform(-jitter * h, jitter * h, size=(int(interior.sum()), 3))
        coords[interior] += d
    return coords


def _cell_origins(nx, ny, nz):
    i, j, k = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    return np.stack([i.ravel(order="F"), j.ravel(order="F"), k.ravel(order="F")], axis=1)


def _node_id(ijk, nx, ny):
    return ijk[..., 0] + (nx + 1) * (ijk[..., 1] + (ny + 1) * ijk[..., 2])


def _coef(n, coef, rng):
    if isinstance(coef, (int, float)):
        return np.full(n, float(coef), dtype=np.float64)
    lo, hi = coef
    return np.exp(rng.uniform(np.log(lo), np.log(hi), size=n))


def box_mesh(
    elem: int,
    nx: int,
    ny: int | None = None,
    nz: int | None = None,
    h: float | None = None,
    jitter: float = 0.0,
    coef=1.0,
    permute_nodes: bool = False,
    permute_elems: bool = False,
    seed: int = 0,
) -> Mesh:
    """Structured box of ``nx*ny*nz`` cells meshed with hex8 or Kuhn tet4.

    ``h`` defaults to ``1/nx`` (so a cube ``nx=ny=nz`` is the unit cube).
    """
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    h = 1.0 / nx if h is None else h
    r_jit, r_nperm, r_eperm, r_coef, _, _ = streams(seed)
    coords = _grid_nodes(nx, ny, nz, h, jitter, r_jit)
    org = _cell_origins(nx, ny, nz)  # [ncell, 3]
    if elem == 8:
        corners = org[:, None, :] + HEX_CORNERS[None, :, :]
        conn = _node_id(corners, nx, ny)
    elif elem == 4:
        blocks = []
        one = np.array([1, 1, 1], dtype=np.int64)
        for p in KUHN_PERMS:
            e0 = np.zeros(3, np.int64)
            e0[p[0]] = 1
            e1 = np.zeros(3, np.int64)
            e1[p[1]] = 1
            v = [org, org + e0, org + e0 + e1, org + one]
            if _perm_is_odd(p):
                v[2], v[3] = v[3], v[2]
            blocks.append(np.stack([_node_id(x, nx, ny) for x in v], axis=1))
        # element id = 6*cell + permutation index
        conn = np.stack(blocks, axis=1).reshape(-1, 4)
    else:
        raise ValueError("elem must be 8 (hex8) or 4 (tet4)")
    nel = conn.shape[0]
    c = _coef(nel, coef, r_coef)
    nn = coords.shape[0]
    if permute_nodes:
        perm = r_nperm.permutation(nn)  # old id -> new id
        conn = perm[conn]
        newc = np.empty_like(coords)
        newc[perm] = coords
        coords = newc
    if permute_elems:
        ep = r_eperm.permutation(nel)
        conn = conn[ep]
        c = c[ep]
    meta = dict(nx=nx, ny=ny, nz=nz, h=h, jitter=jitter, coef=coef, permute_nodes=permute_nodes,
                permute_elems=permute_elems, seed=seed)
    return Mesh(elem, np.ascontiguousarray(conn, dtype=np.int32), np.ascontiguousarray(coords),
                np.ascontiguousarray(c), meta)


# ---------------------------------------------------------------------------
# The five workloads.  ``n`` overrides the cells per axis of the cube configs so
# that the same recipe can be run at sizes an FP64 CPU oracle finishes quickly.
# ---------------------------------------------------------------------------
CONFIG_NAMES = {
    1: "hex8 unit cube 10^3, jitter 0.2h, c=1, FP64",
    2: "hex8 box 100^3, jitter 0.25h, random node numbering, c log-U[1e-2,1e2]",
    3: "tet4 Kuhn 6x150^3, jitter 0.2h, random node+element numbering, c log-U[1e-3,1e3]",
    4: "batch of 256 hex8 boxes, cells per axis U{8..64}, h=1/64, jitter 0.2h, c log-U[1e-2,1e2]",
    5: "hex8 box 64^3, jitter 0.2h, c log-U[1e-1,1e1], FP64 (+ seeded normal loss weights)",
    6: "tet4 Kuhn 6x337^3, jitter 0.2h, c log-U[1e-3,1e3] (more element pairs than one pass indexes)",
    7: "hex8 unit cube 300^3, undistorted, c=1 (the largest mesh of Table 2)",
}
CONFIG_FULL_N = {1: 10, 2: 100, 3: 150, 5: 64, 6: 337, 7: 300}


def config_mesh(cid: int, n: int | None = None) -> Mesh:
    """Mesh of workload ``cid`` (1, 2, 3, 5, 6 or 7); ``n`` shrinks the cube for tests."""
    n = CONFIG_FULL_N[cid] if n is None else n
    if cid == 1:
        return box_mesh(8, n, jitter=0.2, coef=1.0, seed=1)
    if cid == 2:
        return box_mesh(8, n, jitter=0.25, coef=(1e-2, 1e2), permute_nodes=True, seed=2)
    if cid == 3:
        return box_mesh(4, n, jitter=0.2, coef=(1e-3, 1e3), permute_nodes=True, permute_elems=True, seed=3)
    if cid == 5:
        return box_mesh(8, n, jitter=0.2, coef=(1e-1, 1e1), seed=5)
    if cid == 6:
        return box_mesh(4, n, jitter=0.2, coef=(1e-3, 1e3), seed=7)
    if cid == 7:
        return box_mesh(8, n, jitter=0.0, coef=1.0, seed=0)
    raise ValueError(f"config {cid} is not a single mesh")


def config4_batch(n_mesh: int = 256, lo: int = 8, hi: int = 64, seed: int = 4):
    """Workload 4: ``n_mesh`` hex8 boxes with cells per axis i.i.d. U{lo..hi}, h = 1/64."""
    rng = streams(seed, 2)[1]
    dims = rng.integers(lo, hi + 1, size=(n_mesh, 3))
    meshes = []
    for m, (nx, ny, nz) in enumerate(dims):
        meshes.append(box_mesh(8, int(nx), int(ny), int(nz), h=1.0 / 64, jitter=0.2, coef=(1e-2, 1e2),
                               seed=int(np.random.SeedSequence([seed, m]).generate_state(1)[0])))
    return meshes


def loss_weights(n: int, seed: int = 5) -> np.ndarray:
    """Seeded N(0,1) weights on the ``n`` lower-pattern entries (workload 5)."""
    return streams(seed)[4].standard_normal(n)


def counts(elem: int, nx: int, ny: int | None = None, nz: int | None = None):
    """(n_elem, n_node, n_triplets) of a structured box, from the grid sizes alone."""
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    cells = nx * ny * nz
    nel = cells * (1 if elem == 8 else 6)
    nen = elem
    return nel, (nx + 1) * (ny + 1) * (nz + 1), nel * nen * (nen + 1) // 2


def element_matrices(n_elem: int, nd: int, seed: int = 6) -> np.ndarray:
    """Seeded N(0,1) packed lower triangles [n_elem, nd(nd+1)/2] of symmetric element
    matrices (inputs of the assembly-only paths; no physics)."""
    return streams(seed)[5].standard_normal((n_elem, nd * (nd + 1) // 2))


def fan_mesh(n_tets: int, center_last: bool = True, seed: int = 0) -> Mesh:
    """n_tets tets sharing one node (recipe in the module docstring): a node of valence
    n_tets, whose row (centre last) or column (centre first) collects every element."""
    rng = np.random.default_rng(seed)
    nn = 1 + 3 * n_tets
    q = rng.standard_normal((n_tets, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    R = np.stack([np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
                  np.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
                  np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1)], 1)
    corner = np.eye(3)[None] + rng.uniform(-0.2, 0.2, (n_tets, 3, 3))  # rows: the three corners
    scale = rng.uniform(0.5, 2.0, (n_tets, 1, 1))
    X = np.zeros((nn, 3))
    X[1:] = (scale * corner @ np.transpose(R, (0, 2, 1))).reshape(-1, 3)
    t = np.arange(n_tets)
    conn = np.stack([np.zeros(n_tets, np.int64), 1 + 3 * t, 2 + 3 * t, 3 + 3 * t], axis=1)
    if center_last:
        perm = np.roll(np.arange(nn), 1)  # old 0 -> nn-1, old i -> i-1
        newX = np.empty_like(X)
        newX[perm] = X
        conn = perm[conn]
        X = newX
    return Mesh(4, conn.astype(np.int32), X, np.exp(rng.uniform(-2, 2, n_tets)))


def box_nnz(elem: int, nx: int, ny: int, nz: int) -> int:
    """Lower nnz of a structured box: its nodes plus every node pair sharing an element.
    Bricks: axis edges, both diagonals of every face, the four body diagonals of a cell.
    Kuhn tetrahedra: axis edges, one diagonal per face, one body diagonal per cell."""
    X, Y, Z = nx + 1, ny + 1, nz + 1
    axis = nx * Y * Z + X * ny * Z + X * Y * nz
    faces = nx * ny * Z + nx * Y * nz + X * ny * nz
    cells = nx * ny * nz
    if elem == 8:
        return X * Y * Z + axis + 2 * faces + 4 * cells
    return X * Y * Z + axis + faces + cells
