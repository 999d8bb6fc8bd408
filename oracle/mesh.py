"""Two-level finite-volume meshes (Sec. 2.1 of the paper).

The potential phi lives on the fine cells, the density rho and the slack s on
the coarse cells.  Boundary edges are dropped (no-flux condition, Sec. 2.1), so
every edge listed here is interior.

Structured right-triangle grids (the reading used throughout this build)
------------------------------------------------------------------------
The benchmark meshes are the unit square cut into an n x n grid of squares,
each split along its SW-NE diagonal into two right triangles.  A right
triangle's circumcentre is the midpoint of its hypotenuse, so the two
triangles of one square share a circumcentre and the two-point flux distance
across the diagonal is zero.  In the limit of a vanishing distance the two
triangles carry one potential value; the phi-cells are therefore the n^2 fine
squares, each the union of its two triangles.  The density lives on the
(n/2) x (n/2) coarse grid, each coarse square split SW-NE into a lower-right
(LR') and an upper-left (UL') triangle.  Every fine triangle has one coarse
parent triangle, which generalises the 0/1 injection J of Sec. 2.1 to overlap
areas Omega = M J.

Index conventions (shared by every consumer of these meshes):
  fine cell   i = b*n + a          square [a h, (a+1) h] x [b h, (b+1) h]
  coarse cell j = 2*(B*(n/2) + A) + t,  t = 0 for LR' (x >= y), 1 for UL'.

Fine edges: the 2 n (n-1) interior axis-aligned edges, length = distance = h,
lambda = 1/2 (both circumcentres are h/2 from the edge).  Orientation: the
first cell K is the left/bottom one, E(K, e) = +1, E(L, e) = -1.  The density
side of K is the parent of the fine triangle of K that touches the edge.

Coarse edges (used only by the BB approximation of the Schur complement,
Sec. 4.4.3): square legs (length = distance = H) and the diagonal of each
coarse square.  Across the diagonal the circumcentre distance is zero again;
the centroid distance sqrt(2) H / 3 is used instead, so the coarse Laplacian
stays defined.  This only affects the preconditioner, never the solution.

Cartesian meshes
----------------
The paper's Cartesian special case: both levels are the same n x n grid of
squares, J is the identity.  The three-dimensional workload (Sec. 4.1) uses
the n x n x n grid of cubes in the same way, with faces as edges.

Pins (tests/test_oracle_mesh.py): area sums, overlap row/column sums, edge
counts, orientation of the density sides against direct geometric tests.
"""

from __future__ import annotations

import dataclasses
import numpy as np


@dataclasses.dataclass
class Mesh:
    """Generic two-level FV mesh.  All arrays are numpy, float64 / int64."""

    n_fine: int
    n_coarse: int
    fine_area: np.ndarray          # (n_fine,)
    coarse_area: np.ndarray        # (n_coarse,)
    ov_fine: np.ndarray            # overlap entries of Omega = M J
    ov_coarse: np.ndarray
    ov_area: np.ndarray
    fe_K: np.ndarray               # fine edges: cell on the + side
    fe_L: np.ndarray               # cell on the - side
    fe_rK: np.ndarray              # coarse cell feeding R_E on the K side
    fe_rL: np.ndarray              # coarse cell feeding R_E on the L side
    fe_len: np.ndarray
    fe_dist: np.ndarray
    fe_lam: np.ndarray             # weight of the K side in R_E
    ce_i: np.ndarray               # coarse edges (for the BB coarse Laplacian)
    ce_j: np.ndarray
    ce_len: np.ndarray
    ce_dist: np.ndarray
    ce_lam: np.ndarray
    name: str = "mesh"

    @property
    def n_fedge(self) -> int:
        return int(self.fe_K.size)

    @property
    def n_cedge(self) -> int:
        return int(self.ce_i.size)

    @property
    def domain_area(self) -> float:
        return float(self.coarse_area.sum())


def _coarse_index(n: int, A: int, B: int, t: int) -> int:
    return 2 * (B * (n // 2) + A) + t


def _parents(n: int, a: int, b: int):
    """Coarse parents of the (LR, UL) fine triangles of fine square (a, b).

    Local position (a mod 2, b mod 2) inside the coarse square:
      (1,0): the square lies below the coarse diagonal -> both halves in LR'
      (0,1): the square lies above it                  -> both halves in UL'
      (0,0), (1,1): the coarse diagonal is the square's own diagonal,
                    LR -> LR', UL -> UL'.
    """
    A, B = a // 2, b // 2
    la, lb = a % 2, b % 2
    lr = _coarse_index(n, A, B, 1 if (la, lb) == (0, 1) else 0)
    ul = _coarse_index(n, A, B, 0 if (la, lb) == (1, 0) else 1)
    return lr, ul


def structured_mesh(n: int) -> Mesh:
    """Two-level mesh of the n x n right-triangle grid (module docstring)."""
    if n < 2 or n % 2:
        raise ValueError("n must be even and >= 2")
    h = 1.0 / n
    H = 2.0 * h
    nc = n // 2
    n_fine = n * n
    n_coarse = 2 * nc * nc

    fine_area = np.full(n_fine, h * h)
    coarse_area = np.full(n_coarse, 2.0 * h * h)

    ov = {}
    for b in range(n):
        for a in range(n):
            i = b * n + a
            lr, ul = _parents(n, a, b)
            ov[(i, lr)] = ov.get((i, lr), 0.0) + 0.5 * h * h
            ov[(i, ul)] = ov.get((i, ul), 0.0) + 0.5 * h * h
    keys = sorted(ov)
    ov_fine = np.array([k[0] for k in keys], dtype=np.int64)
    ov_coarse = np.array([k[1] for k in keys], dtype=np.int64)
    ov_area = np.array([ov[k] for k in keys])

    K, L, rK, rL = [], [], [], []
    # vertical edges x = (a+1) h between squares (a, b) and (a+1, b):
    # the right side of (a, b) belongs to its LR triangle, the left side of
    # (a+1, b) to its UL triangle.
    for b in range(n):
        for a in range(n - 1):
            K.append(b * n + a)
            L.append(b * n + a + 1)
            rK.append(_parents(n, a, b)[0])
            rL.append(_parents(n, a + 1, b)[1])
    # horizontal edges y = (b+1) h between (a, b) and (a, b+1): the top of
    # (a, b) belongs to its UL triangle, the bottom of (a, b+1) to its LR one.
    for b in range(n - 1):
        for a in range(n):
            K.append(b * n + a)
            L.append((b + 1) * n + a)
            rK.append(_parents(n, a, b)[1])
            rL.append(_parents(n, a, b + 1)[0])
    ne = len(K)
    fe_len = np.full(ne, h)
    fe_dist = np.full(ne, h)
    fe_lam = np.full(ne, 0.5)

    ci, cj, cl, cd = [], [], [], []
    for B in range(nc):
        for A in range(nc):
            # diagonal of the coarse square: centroid distance (module doc)
            ci.append(_coarse_index(n, A, B, 0))
            cj.append(_coarse_index(n, A, B, 1))
            cl.append(np.sqrt(2.0) * H)
            cd.append(np.sqrt(2.0) * H / 3.0)
    for B in range(nc):
        for A in range(nc - 1):
            # vertical leg: LR' of (A, B) touches x = (A+1) H, UL' of (A+1, B)
            ci.append(_coarse_index(n, A, B, 0))
            cj.append(_coarse_index(n, A + 1, B, 1))
            cl.append(H)
            cd.append(H)
    for B in range(nc - 1):
        for A in range(nc):
            # horizontal leg: UL' of (A, B) touches y = (B+1) H, LR' of (A, B+1)
            ci.append(_coarse_index(n, A, B, 1))
            cj.append(_coarse_index(n, A, B + 1, 0))
            cl.append(H)
            cd.append(H)

    return Mesh(
        n_fine=n_fine, n_coarse=n_coarse,
        fine_area=fine_area, coarse_area=coarse_area,
        ov_fine=ov_fine, ov_coarse=ov_coarse, ov_area=ov_area,
        fe_K=np.array(K, dtype=np.int64), fe_L=np.array(L, dtype=np.int64),
        fe_rK=np.array(rK, dtype=np.int64), fe_rL=np.array(rL, dtype=np.int64),
        fe_len=fe_len, fe_dist=fe_dist, fe_lam=fe_lam,
        ce_i=np.array(ci, dtype=np.int64), ce_j=np.array(cj, dtype=np.int64),
        ce_len=np.array(cl), ce_dist=np.array(cd),
        ce_lam=np.full(len(ci), 0.5),
        name=f"structured{n}",
    )


def cartesian_mesh(n: int) -> Mesh:
    """Single n x n Cartesian grid for both levels (J = identity)."""
    if n < 2:
        raise ValueError("n must be >= 2")
    h = 1.0 / n
    N = n * n
    K, L = [], []
    for b in range(n):
        for a in range(n - 1):
            K.append(b * n + a)
            L.append(b * n + a + 1)
    for b in range(n - 1):
        for a in range(n):
            K.append(b * n + a)
            L.append((b + 1) * n + a)
    K = np.array(K, dtype=np.int64)
    L = np.array(L, dtype=np.int64)
    ne = K.size
    return Mesh(
        n_fine=N, n_coarse=N,
        fine_area=np.full(N, h * h), coarse_area=np.full(N, h * h),
        ov_fine=np.arange(N, dtype=np.int64), ov_coarse=np.arange(N, dtype=np.int64),
        ov_area=np.full(N, h * h),
        fe_K=K, fe_L=L, fe_rK=K.copy(), fe_rL=L.copy(),
        fe_len=np.full(ne, h), fe_dist=np.full(ne, h), fe_lam=np.full(ne, 0.5),
        ce_i=K.copy(), ce_j=L.copy(), ce_len=np.full(ne, h), ce_dist=np.full(ne, h),
        ce_lam=np.full(ne, 0.5),
        name=f"cartesian{n}",
    )


def cartesian3d_mesh(n: int) -> Mesh:
    """n x n x n grid of cubes on [0,1]^3 for both levels (J = identity): the
    three-dimensional workload of Sec. 4.1 (fourth test case).

    Cell i = (c n + b) n + a is the cube [a h, (a+1) h] x [b h, (b+1) h] x
    [c h, (c+1) h], h = 1/n.  The TPFA "edges" of Sec. 2.1 are the interior
    faces: |e| = h^2 (face area), d_e = h (distance of the cell centres),
    lambda_e = 1/2; K is the cell with the smaller coordinate along the
    face normal.  "Areas" are cell volumes h^3.  The coarse edges of the BB
    coarse Laplacian are the same faces.
    """
    if n < 2:
        raise ValueError("n must be >= 2")
    h = 1.0 / n
    N = n ** 3
    idx = np.arange(N, dtype=np.int64).reshape(n, n, n)     # [c, b, a]
    K = np.concatenate([idx[:, :, :-1].ravel(), idx[:, :-1, :].ravel(), idx[:-1, :, :].ravel()])
    L = np.concatenate([idx[:, :, 1:].ravel(), idx[:, 1:, :].ravel(), idx[1:, :, :].ravel()])
    ne = K.size
    return Mesh(
        n_fine=N, n_coarse=N,
        fine_area=np.full(N, h ** 3), coarse_area=np.full(N, h ** 3),
        ov_fine=np.arange(N, dtype=np.int64), ov_coarse=np.arange(N, dtype=np.int64),
        ov_area=np.full(N, h ** 3),
        fe_K=K, fe_L=L, fe_rK=K.copy(), fe_rL=L.copy(),
        fe_len=np.full(ne, h * h), fe_dist=np.full(ne, h), fe_lam=np.full(ne, 0.5),
        ce_i=K.copy(), ce_j=L.copy(), ce_len=np.full(ne, h * h), ce_dist=np.full(ne, h),
        ce_lam=np.full(ne, 0.5),
        name=f"cartesian3d_{n}",
    )


def mesh_from_arrays(d, name="generic") -> Mesh:
    """Oracle Mesh from the arrays of a generic mesh description."""
    fe = np.asarray(d["fe_cell"], dtype=np.int64).reshape(-1, 2)
    fr = np.asarray(d["fe_rho"], dtype=np.int64).reshape(-1, 2)
    ce = np.asarray(d["ce_cell"], dtype=np.int64).reshape(-1, 2)
    return Mesh(
        n_fine=len(d["fine_area"]), n_coarse=len(d["coarse_area"]),
        fine_area=np.asarray(d["fine_area"], float), coarse_area=np.asarray(d["coarse_area"], float),
        ov_fine=np.asarray(d["ov_fine"], np.int64), ov_coarse=np.asarray(d["ov_coarse"], np.int64),
        ov_area=np.asarray(d["ov_area"], float),
        fe_K=fe[:, 0].copy(), fe_L=fe[:, 1].copy(), fe_rK=fr[:, 0].copy(), fe_rL=fr[:, 1].copy(),
        fe_len=np.asarray(d["fe_len"], float), fe_dist=np.asarray(d["fe_dist"], float),
        fe_lam=np.asarray(d["fe_lambda"], float),
        ce_i=ce[:, 0].copy(), ce_j=ce[:, 1].copy(), ce_len=np.asarray(d["ce_len"], float),
        ce_dist=np.asarray(d["ce_dist"], float), ce_lam=np.asarray(d["ce_lambda"], float),
        name=name)
