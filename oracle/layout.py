"""User-facing ordering of unknowns and boundary data, written independently
from the C header's definition.  Test infrastructure only.

Definition (as documented for fds_plan_create):
* Rectangles are closed node boxes (i0, j0, i1, j1).  The coupled subdomains
  are the rectangles that share an edge with two or more others; when there is
  none, the coupled subdomain (the "centre") is the rectangle that shares an
  edge with the largest number of others, ties going to the first listed.
* A rectangle owns its interior nodes.  The nodes strictly inside an edge
  shared by a coupled and a non-coupled rectangle belong to the non-coupled
  one; those strictly inside an edge shared by two coupled rectangles belong
  to the one listed first.
* The unknown vector lists, rectangle by rectangle in the given order, the
  owned nodes in row-major order (j ascending outer, i ascending inner).
* The Dirichlet data vector lists, rectangle by rectangle, the values on the
  rectangle's whole closed box in row-major order; only entries at Dirichlet
  nodes are read.
"""

from __future__ import annotations

from typing import List, Sequence, Tuple

import numpy as np

Rect = Tuple[int, int, int, int]


def _share_edge(a: Rect, b: Rect) -> bool:
    ai0, aj0, ai1, aj1 = a
    bi0, bj0, bi1, bj1 = b
    if ai1 == bi0 or ai0 == bi1:
        return min(aj1, bj1) - max(aj0, bj0) > 0
    if aj1 == bj0 or aj0 == bj1:
        return min(ai1, bi1) - max(ai0, bi0) > 0
    return False


def coupled_indices(rects: Sequence[Rect]) -> List[int]:
    counts = [sum(_share_edge(a, b) for b in rects if b is not a) for a in rects]
    several = [r for r, k in enumerate(counts) if k >= 2]
    if several:
        return several
    return [counts.index(max(counts))]


def centre_index(rects: Sequence[Rect]) -> int:
    """The single coupled rectangle (geometries with one coupled subdomain)."""
    cs = coupled_indices(rects)
    if len(cs) != 1:
        raise ValueError("geometry has several coupled subdomains")
    return cs[0]


def _edge_owner(rects: Sequence[Rect], coupled: Sequence[int], r: int, q: int) -> int:
    if (r in coupled) != (q in coupled):
        return q if r in coupled else r
    return min(r, q)


def owned_nodes(rects: Sequence[Rect]) -> List[Tuple[np.ndarray, np.ndarray]]:
    """For each rectangle, (j, i) index arrays of its owned nodes in order."""
    coupled = coupled_indices(rects)
    out = []
    for r, (i0, j0, i1, j1) in enumerate(rects):
        ilo, ihi, jlo, jhi = i0 + 1, i1 - 1, j0 + 1, j1 - 1   # inclusive interior
        for q, other in enumerate(rects):
            if q == r or not _share_edge(rects[r], other):
                continue
            if _edge_owner(rects, coupled, r, q) != r:
                continue
            oi0, oj0, oi1, oj1 = other
            if i0 == oi1:
                ilo = i0        # owns its west edge
            elif i1 == oi0:
                ihi = i1        # owns its east edge
            elif j0 == oj1:
                jlo = j0        # owns its south edge
            elif j1 == oj0:
                jhi = j1        # owns its north edge
        jj, ii = np.meshgrid(np.arange(jlo, jhi + 1), np.arange(ilo, ihi + 1), indexing="ij")
        out.append((jj.ravel(), ii.ravel()))
    return out


def block_shapes(rects: Sequence[Rect]) -> List[Tuple[int, int]]:
    """(rows, cols) of each rectangle's owned block."""
    shapes = []
    for jj, ii in owned_nodes(rects):
        shapes.append((len(np.unique(jj)), len(np.unique(ii))))
    return shapes


def to_user(rects: Sequence[Rect], grid_values: np.ndarray) -> np.ndarray:
    parts = [np.asarray(grid_values)[jj, ii] for jj, ii in owned_nodes(rects)]
    return np.concatenate(parts).astype(np.float64)


def from_user(rects: Sequence[Rect], vec: np.ndarray, shape: Tuple[int, int],
              fill=np.nan) -> np.ndarray:
    out = np.full(shape, fill, dtype=np.float64)
    k = 0
    for jj, ii in owned_nodes(rects):
        out[jj, ii] = vec[k:k + len(jj)]
        k += len(jj)
    return out


def bc_boxes(rects: Sequence[Rect], g_grid: np.ndarray) -> np.ndarray:
    parts = [np.asarray(g_grid)[j0:j1 + 1, i0:i1 + 1].ravel() for (i0, j0, i1, j1) in rects]
    return np.concatenate(parts).astype(np.float64)
