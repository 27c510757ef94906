"""Host-side packing of whole-frame fields into the C ABI's user layout.

The ABI takes, per rectangle in plan order, (a) the owned unknown nodes in
row-major order and (b) the values on the rectangle's closed box (Dirichlet
data).  These helpers cut those blocks out of arrays defined on all nodes of
a bounding grid (array[j, i] = value at node (i, j)).  Pure indexing.
"""

from __future__ import annotations

from typing import List, Sequence, Tuple

import numpy as np

Rect = Tuple[int, int, int, int]


def _touches(a, b) -> bool:
    if a[2] == b[0] or a[0] == b[2]:
        return min(a[3], b[3]) - max(a[1], b[1]) > 0
    if a[3] == b[1] or a[1] == b[3]:
        return min(a[2], b[2]) - max(a[0], b[0]) > 0
    return False


def _coupled(rects: Sequence[Rect]) -> List[int]:
    """Indices of the coupled rectangles: those touching two or more others,
    else the first of those touching the most."""
    deg = [sum(_touches(a, b) for k, b in enumerate(rects) if k != r) for r, a in enumerate(rects)]
    out = [r for r, d in enumerate(deg) if d >= 2]
    return out if out else [int(np.argmax(deg))]


def owned_box(rects: Sequence[Rect], r: int) -> Tuple[int, int, int, int]:
    """Inclusive (ilo, ihi, jlo, jhi) node ranges owned by rectangle r: its
    interior, plus for a non-coupled rectangle the line it shares with the
    coupled block, plus for a coupled rectangle each line it shares with a
    coupled rectangle listed after it."""
    coupled = _coupled(rects)
    i0, j0, i1, j1 = rects[r]
    ilo, ihi, jlo, jhi = i0 + 1, i1 - 1, j0 + 1, j1 - 1
    if r in coupled:
        for q in coupled:
            if q <= r or not _touches(rects[r], rects[q]):
                continue
            qi0, qj0, qi1, qj1 = rects[q]
            if qi1 == i0:
                ilo = i0
            elif qi0 == i1:
                ihi = i1
            elif qj1 == j0:
                jlo = j0
            elif qj0 == j1:
                jhi = j1
        return ilo, ihi, jlo, jhi
    for q in coupled:
        if not _touches(rects[r], rects[q]):
            continue
        qi0, qj0, qi1, qj1 = rects[q]
        if i0 == qi1:
            ilo = i0
        elif i1 == qi0:
            ihi = i1
        elif j0 == qj1:
            jlo = j0
        elif j1 == qj0:
            jhi = j1
        break
    return ilo, ihi, jlo, jhi


def pack_unknowns(rects: Sequence[Rect], grid: np.ndarray) -> np.ndarray:
    parts = []
    for r in range(len(rects)):
        ilo, ihi, jlo, jhi = owned_box(rects, r)
        parts.append(np.asarray(grid)[jlo:jhi + 1, ilo:ihi + 1].ravel())
    return np.ascontiguousarray(np.concatenate(parts), dtype=np.float64)


def unpack_unknowns(rects: Sequence[Rect], vec: np.ndarray, shape) -> np.ndarray:
    out = np.full(shape, np.nan)
    k = 0
    for r in range(len(rects)):
        ilo, ihi, jlo, jhi = owned_box(rects, r)
        h, w = jhi - jlo + 1, ihi - ilo + 1
        out[jlo:jhi + 1, ilo:ihi + 1] = np.asarray(vec[k:k + h * w]).reshape(h, w)
        k += h * w
    return out


def pack_boxes(rects: Sequence[Rect], grid: np.ndarray) -> np.ndarray:
    parts = [np.asarray(grid)[j0:j1 + 1, i0:i1 + 1].ravel() for (i0, j0, i1, j1) in rects]
    return np.ascontiguousarray(np.concatenate(parts), dtype=np.float64)
