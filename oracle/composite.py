"""Global composite-grid 5-point system: assembly and direct solve (FP64).

Test infrastructure only (see the package docstring).

Definitions (Section 2.1, central-difference scheme; Section 2.3, block system;
Introduction, model equation  lap(p) + kappa p = f):

* The domain is the union of closed axis-aligned rectangles whose corners are
  grid nodes.  A grid cell (the unit box with lower-left node (i, j)) belongs to
  the domain when it lies inside one of the rectangles.
* A node is an UNKNOWN when all four cells that touch it belong to the domain
  (it is an interior point of the union).  Nodes strictly inside a shared edge
  between two rectangles are unknowns by this rule.
* A node of the closed domain that is not an unknown is a DIRICHLET node; its
  value is taken from the boundary data g.
* Row of the unknown at (i, j):
      delta*(p[i+1,j] + p[i-1,j] + p[i,j+1] + p[i,j-1]) + (kappa - 4 delta) p[i,j] = f[i,j]
  with delta = 1/h^2 (uniform spacing); Dirichlet neighbours move to the right
  side as  -delta*g.
* Unknowns are numbered row-major over the bounding box (j outer, i inner), so
  the matrix is banded with half-bandwidth equal to the widest jump between
  vertically adjacent unknowns.
"""

from __future__ import annotations

import os
from dataclasses import dataclass
from typing import List, Sequence, Tuple

import numpy as np
import scipy.linalg
import scipy.sparse as sp
import scipy.sparse.linalg as spla

Rect = Tuple[int, int, int, int]


@dataclass
class Grid:
    """Node classification of a composite domain on its bounding box."""
    width: int            # number of node columns (I + 1)
    height: int           # number of node rows (J + 1)
    unknown: np.ndarray   # bool (height, width)
    dirichlet: np.ndarray  # bool (height, width)
    index: np.ndarray     # int64 (height, width), -1 where not an unknown

    @property
    def n_unknowns(self) -> int:
        return int(self.unknown.sum())


def classify(rects: Sequence[Rect]) -> Grid:
    I = max(r[2] for r in rects)
    J = max(r[3] for r in rects)
    cells = np.zeros((J, I), dtype=bool)          # cell (j, i): [i, i+1] x [j, j+1]
    for (i0, j0, i1, j1) in rects:
        if not (i1 > i0 and j1 > j0):
            raise ValueError("degenerate rectangle")
        cells[j0:j1, i0:i1] = True
    # pad so every node has four neighbouring cells
    c = np.zeros((J + 2, I + 2), dtype=bool)
    c[1:-1, 1:-1] = cells
    # node (j, i) touches cells (j-1,i-1), (j-1,i), (j,i-1), (j,i) -> padded +1
    ll = c[0:J + 1, 0:I + 1]
    lr = c[0:J + 1, 1:I + 2]
    ul = c[1:J + 2, 0:I + 1]
    ur = c[1:J + 2, 1:I + 2]
    unknown = ll & lr & ul & ur
    closed = ll | lr | ul | ur
    dirichlet = closed & ~unknown
    index = np.full(unknown.shape, -1, dtype=np.int64)
    index[unknown] = np.arange(int(unknown.sum()), dtype=np.int64)
    return Grid(I + 1, J + 1, unknown, dirichlet, index)


def assemble(rects: Sequence[Rect], h: float, kappa: float, f_grid: np.ndarray,
             g_grid: np.ndarray):
    """Return (A csr, b, grid).  f_grid and g_grid cover at least the bounding
    box: f_grid[j, i] is the source at node (i, j), g_grid[j, i] the Dirichlet
    value there."""
    grid = classify(rects)
    H, W = grid.height, grid.width
    f = np.asarray(f_grid, dtype=np.float64)[:H, :W]
    g = np.asarray(g_grid, dtype=np.float64)[:H, :W]
    delta = 1.0 / (h * h)
    jj, ii = np.nonzero(grid.unknown)
    rows_u = grid.index[jj, ii]
    b = f[jj, ii].copy()
    rows = [rows_u]
    cols = [rows_u]
    vals = [np.full(rows_u.shape, kappa - 4.0 * delta)]
    for dj, di in ((0, 1), (0, -1), (1, 0), (-1, 0)):
        nj, ni = jj + dj, ii + di
        nb_unknown = grid.unknown[nj, ni]
        nb_dir = grid.dirichlet[nj, ni]
        if not np.all(nb_unknown | nb_dir):
            raise AssertionError("an unknown has a neighbour outside the closed domain")
        sel = nb_unknown
        rows.append(rows_u[sel])
        cols.append(grid.index[nj[sel], ni[sel]])
        vals.append(np.full(int(sel.sum()), delta))
        sel = nb_dir
        np.subtract.at(b, rows_u[sel], delta * g[nj[sel], ni[sel]])
    nu = grid.n_unknowns
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(nu, nu))
    A.sum_duplicates()
    return A, b, grid


def half_bandwidth(A: sp.spmatrix) -> int:
    c = A.tocoo()
    return int(np.max(np.abs(c.row - c.col))) if c.nnz else 0


def band_solve(A: sp.spmatrix, b: np.ndarray, spd_negative: bool) -> np.ndarray:
    """Direct banded solve.  If -A is symmetric positive definite, LAPACK banded
    Cholesky (pbsv) on -A; otherwise LAPACK banded LU with partial pivoting
    (gbsv)."""
    c = A.tocoo()
    n = A.shape[0]
    bw = half_bandwidth(A)
    if spd_negative:
        lower = c.row >= c.col
        ab = np.zeros((bw + 1, n))
        ab[(c.row - c.col)[lower], c.col[lower]] = -c.data[lower]
        return scipy.linalg.solveh_banded(ab, -b, lower=True, check_finite=False)
    ab = np.zeros((2 * bw + 1, n))
    ab[bw + c.row - c.col, c.col] = c.data
    return scipy.linalg.solve_banded((bw, bw), ab, b, check_finite=False)


def sparse_lu(A: sp.spmatrix):
    """SuperLU factorisation of the assembled matrix.  The column order is a
    minimum-degree order of the pattern of A + A^T, which suits the symmetric
    5-point matrix (about half the fill of the default column order)."""
    return spla.splu(A.tocsc(), permc_spec="MMD_AT_PLUS_A")


def sparse_lu_solve(A: sp.spmatrix, b: np.ndarray) -> np.ndarray:
    """SuperLU on the same assembled matrix (used where a dense band would not
    fit in host memory)."""
    return sparse_lu(A).solve(b)


BAND_BYTES_LIMIT = int(os.environ.get("FDS_ORACLE_BAND_BYTES", str(6 << 30)))


@dataclass
class Solution:
    p: np.ndarray          # values at unknowns, in grid index order
    grid: Grid
    relres: float          # ||b - A p||_2 / ||b||_2 in FP64
    method: str

    def on_grid(self, fill=np.nan) -> np.ndarray:
        out = np.full((self.grid.height, self.grid.width), fill)
        out[self.grid.unknown] = self.p
        return out


def solve(rects: Sequence[Rect], h: float, kappa: float, f_grid, g_grid,
          method: str = "auto") -> Solution:
    """Direct FP64 solution of the composite system (the oracle answer)."""
    A, b, grid = assemble(rects, h, kappa, f_grid, g_grid)
    n = A.shape[0]
    bw = half_bandwidth(A)
    if method == "auto":
        method = "band" if (bw + 1) * n * 8 <= BAND_BYTES_LIMIT else "splu"
    if method == "band":
        p = band_solve(A, b, spd_negative=(kappa <= 0.0))
    elif method == "band_lu":
        p = band_solve(A, b, spd_negative=False)
    elif method == "splu":
        p = sparse_lu_solve(A, b)
    elif method == "dense":
        p = np.linalg.solve(A.toarray(), b)
    else:
        raise ValueError(method)
    r = b - A @ p
    nb = np.linalg.norm(b)
    return Solution(p, grid, float(np.linalg.norm(r) / nb) if nb > 0 else 0.0, method)


def solve_many(rects: Sequence[Rect], h: float, kappa: float, fg: Sequence[Tuple[np.ndarray, np.ndarray]],
               method: str = "auto") -> List[Solution]:
    """solve() for several (f_grid, g_grid) pairs on one domain: the matrix is
    assembled and factorised once (the right-hand sides differ)."""
    if not fg:
        return []
    A, b0, grid = assemble(rects, h, kappa, fg[0][0], fg[0][1])
    bs = [b0] + [assemble(rects, h, kappa, f, g)[1] for (f, g) in fg[1:]]
    n = A.shape[0]
    bw = half_bandwidth(A)
    if method == "auto":
        method = "band" if (bw + 1) * n * 8 <= BAND_BYTES_LIMIT else "splu"
    out = []
    if method == "splu":
        lu = sparse_lu(A)
        ps = [lu.solve(b) for b in bs]
    elif method == "band":
        ps = [band_solve(A, b, spd_negative=(kappa <= 0.0)) for b in bs]
    else:
        raise ValueError(method)
    for p, b in zip(ps, bs):
        nb = np.linalg.norm(b)
        out.append(Solution(p, grid, float(np.linalg.norm(b - A @ p) / nb) if nb > 0 else 0.0, method))
    return out


def residual(rects: Sequence[Rect], h: float, kappa: float, f_grid, g_grid,
             p_unknowns: np.ndarray) -> float:
    """||b - A p||_2 / ||b||_2 of any candidate p (unknown order)."""
    A, b, _ = assemble(rects, h, kappa, f_grid, g_grid)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(b - A @ p_unknowns) / nb) if nb > 0 else 0.0
