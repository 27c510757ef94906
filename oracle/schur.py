"""Schur-complement view of the composite system and a reference GMRES.

Test infrastructure only (see the package docstring).

Section 2.3: ordering the unknowns by subdomain gives a block system with
diagonal blocks A_i and interface couplings R_ij = R_ji^T.  Eliminating every
subdomain except the coupled one leaves  L_c p_c = f'_c  with
    L_c  = A_cc - sum_a R_ca A_a^{-1} R_ac,
    f'_c = f_c  - sum_a R_ca A_a^{-1} f_a.
Here these blocks are cut straight out of the assembled global matrix (no
transforms, no closed forms), which is the plain definition.

Section 2.4: GMRES on the interface system, preconditioned by A_cc^{-1}
(the block operator without the Schur complement).  The paper calls it a right
preconditioner; `gmres_right` follows the listed steps -- Arnoldi with
Gram-Schmidt (modified form), the Hessenberg least-squares problem solved by
Givens rotations, the update, the tolerance test -- in that order.
"""

from __future__ import annotations

from dataclasses import dataclass
from typing import Callable, List, Optional, Sequence, Tuple

import numpy as np
import scipy.linalg
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import composite, layout


@dataclass
class Partition:
    A: sp.csr_matrix
    b: np.ndarray
    centre: np.ndarray          # global unknown indices of the centre, centre row-major order
    arms: List[np.ndarray]      # global unknown indices of each other rectangle (user order)
    centre_shape: Tuple[int, int]
    rest: np.ndarray            # all non-centre unknowns

    def block(self, r, c):
        return self.A[r][:, c]


def partition(rects, h, kappa, f_grid, g_grid) -> Partition:
    A, b, grid = composite.assemble(rects, h, kappa, f_grid, g_grid)
    own = layout.owned_nodes(rects)
    c = layout.centre_index(rects)
    idx = [grid.index[jj, ii] for jj, ii in own]
    assert all((x >= 0).all() for x in idx)
    rest = np.concatenate([idx[r] for r in range(len(rects)) if r != c]) if len(rects) > 1 \
        else np.zeros(0, dtype=np.int64)
    shapes = layout.block_shapes(rects)
    return Partition(A, b, idx[c], [idx[r] for r in range(len(rects)) if r != c],
                     shapes[c], rest)


class SchurOperator:
    """Applies L_c, A_cc^{-1} and forms f'_c by sparse direct solves."""

    def __init__(self, P: Partition):
        self.P = P
        A = P.A
        C, R = P.centre, P.rest
        self.Acc = A[C][:, C].tocsc()
        self.Acc_lu = spla.splu(self.Acc)
        if len(R):
            self.Acr = A[C][:, R].tocsr()
            self.Arc = A[R][:, C].tocsr()
            self.Arr_lu = spla.splu(A[R][:, R].tocsc())
        else:
            self.Acr = self.Arc = self.Arr_lu = None

    def schur_apply(self, z):
        """S z = A_cr A_rr^{-1} A_rc z (zero for a single rectangle)."""
        if self.Acr is None:
            return np.zeros_like(z)
        return self.Acr @ self.Arr_lu.solve(self.Arc @ z)

    def apply_L(self, z):
        return self.Acc @ z - self.schur_apply(z)

    def apply_Minv(self, v):
        return self.Acc_lu.solve(np.asarray(v, dtype=np.float64))

    def fprime(self):
        bC = self.P.b[self.P.centre]
        if self.Acr is None:
            return bC.copy()
        return bC - self.Acr @ self.Arr_lu.solve(self.P.b[self.P.rest])

    def back_substitute(self, pc):
        """Arm values from the centre values: p_R = A_rr^{-1}(b_R - A_rc p_c)."""
        if self.Acr is None:
            return np.zeros(0)
        return self.Arr_lu.solve(self.P.b[self.P.rest] - self.Arc @ pc)

    def jacobi_diagonal(self):
        """diag(L_c) = diag(A_cc) - diag(S) (Section 3.2's Jacobi
        preconditioner), from the assembled blocks: S e_b is nonzero only for
        the centre nodes b that couple to another subdomain, so one solve per
        such node gives diag(S)."""
        d = np.asarray(self.Acc.diagonal(), dtype=np.float64).copy()
        if self.Acr is None:
            return d
        Arc = self.Arc.tocsc()
        B = np.flatnonzero(np.diff(Arc.indptr))
        if B.size:
            X = self.Arr_lu.solve(Arc[:, B].toarray())
            Y = self.Acr[B, :] @ X
            d[B] -= np.diag(np.asarray(Y))
        return d

    def apply_Jinv(self, v):
        if not hasattr(self, "_jd"):
            self._jd = self.jacobi_diagonal()
        return np.asarray(v, dtype=np.float64) / self._jd

    def dense_L(self):
        n = self.Acc.shape[0]
        return np.column_stack([self.apply_L(e) for e in np.eye(n)])

    def dense_S(self):
        n = self.Acc.shape[0]
        return np.column_stack([self.schur_apply(e) for e in np.eye(n)])


def arm_schur_block(P: Partition, arm: int) -> np.ndarray:
    """Dense S_ca = R_ca A_a^{-1} R_ac for one arm, restricted to the centre."""
    A = P.A
    C, a = P.centre, P.arms[arm]
    Aca = A[C][:, a].toarray()
    Aac = A[a][:, C].toarray()
    Aaa = A[a][:, a].toarray()
    return Aca @ np.linalg.solve(Aaa, Aac)


# --------------------------------------------------------------------------- Krylov pieces

def mgs_step(V: np.ndarray, w: np.ndarray):
    """One Arnoldi step with modified Gram-Schmidt: V holds j+1 orthonormal
    rows; returns (h of length j+2, v_next)."""
    w = np.array(w, dtype=np.float64, copy=True)
    k = V.shape[0]
    h = np.zeros(k + 1)
    for i in range(k):
        h[i] = np.dot(w, V[i])
        w -= h[i] * V[i]
    h[k] = np.linalg.norm(w)
    return h, (w / h[k] if h[k] > 0 else w)


def givens(a: float, b: float):
    """Rotation (c, s) with c a + s b = rho, -s a + c b = 0, rho = hypot(a, b)."""
    rho = np.hypot(a, b)
    if rho == 0.0:
        return 1.0, 0.0, 0.0
    return a / rho, b / rho, rho


@dataclass
class GmresResult:
    x: np.ndarray
    iterations: int
    cycles: int
    relres: float
    history: List[float]
    converged: bool


def gmres_right(apply_L: Callable, apply_Minv: Callable, f: np.ndarray, m: int, tol: float,
                max_cycles: int = 200, x0: Optional[np.ndarray] = None) -> GmresResult:
    f = np.asarray(f, dtype=np.float64)
    nf = np.linalg.norm(f)
    x = np.zeros_like(f) if x0 is None else np.array(x0, dtype=np.float64)
    r = f - apply_L(x) if x0 is not None else f.copy()
    beta = np.linalg.norm(r)
    hist = [beta / nf if nf > 0 else 0.0]
    its = 0
    if nf == 0.0:
        return GmresResult(x, 0, 0, 0.0, hist, True)
    for cyc in range(1, max_cycles + 1):
        if beta / nf <= tol:
            return GmresResult(x, its, cyc - 1, beta / nf, hist, True)
        V = np.zeros((m + 1, f.size))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        V[0] = r / beta
        g[0] = beta
        k = 0
        for j in range(m):
            w = apply_L(apply_Minv(V[j]))
            for i in range(j + 1):
                H[i, j] = np.dot(w, V[i])
                w -= H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            breakdown = H[j + 1, j] <= 1e-14 * beta
            if not breakdown:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
                a, b = H[i, j], H[i + 1, j]
                H[i, j] = cs[i] * a + sn[i] * b
                H[i + 1, j] = -sn[i] * a + cs[i] * b
            c, s, rho = givens(H[j, j], H[j + 1, j])
            cs[j], sn[j] = c, s
            H[j, j] = rho
            H[j + 1, j] = 0.0
            g[j + 1] = -s * g[j]
            g[j] = c * g[j]
            its += 1
            k = j + 1
            hist.append(abs(g[j + 1]) / nf)
            if abs(g[j + 1]) / nf <= tol or breakdown:
                break
        y = scipy.linalg.solve_triangular(H[:k, :k], g[:k])
        x = x + apply_Minv(V[:k].T @ y)
        r = f - apply_L(x)
        beta = np.linalg.norm(r)
    return GmresResult(x, its, max_cycles, beta / nf, hist, beta / nf <= tol)
