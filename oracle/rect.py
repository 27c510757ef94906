"""Single-rectangle pieces of the fast solver, written as plain definitions.

Test infrastructure only (see the package docstring).

Section 2.1 of the paper: on a rectangle with zero Dirichlet data the 5-point
operator is block tridiagonal; the line matrix is symmetric Toeplitz and is
diagonalised by the sine transform whose eigenvectors are
sqrt(2/(n+1)) sin(j k pi/(n+1)); its eigenvalues have the closed form
-2(dx + dy) + 2 dy cos(k pi/(n+1)).  After the transform every mode k obeys an
independent tridiagonal system with off-diagonal dx and diagonal lambda_k.

Everything here is the dense / banded definition of those objects.  The HIP
path computes the same results with fast transforms and recurrences.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg
import scipy.sparse as sp


# --------------------------------------------------------------------------- DST-I

def dst1_matrix(n: int) -> np.ndarray:
    """S[j-1, k-1] = sin(pi j k / (n+1)), j, k = 1..n (unnormalised DST-I).

    sin(pi t/(n+1)) has period 2(n+1) in the integer t = j k, so t is reduced
    modulo 2(n+1) in exact integer arithmetic before the angle is formed;
    otherwise the rounding of pi*t/(n+1) (t up to n^2) would perturb entries
    by about 1e-12 at n = 2048."""
    j = np.arange(1, n + 1, dtype=np.int64)
    t = np.outer(j, j) % (2 * (n + 1))
    return np.sin(np.pi * t.astype(np.float64) / (n + 1))


def dst1_rows(x: np.ndarray) -> np.ndarray:
    """Unnormalised DST-I of every row: X[r, k] = sum_j x[r, j] sin(pi j k/(n+1))."""
    x = np.asarray(x, dtype=np.float64)
    return x @ dst1_matrix(x.shape[-1])


def sine_eigvecs(n: int) -> np.ndarray:
    """Orthonormal eigenvector matrix Q_D of the Dirichlet line matrix."""
    return np.sqrt(2.0 / (n + 1)) * dst1_matrix(n)


def line_matrix(n: int, dx: float, dy: float) -> np.ndarray:
    """Dirichlet line matrix A_y^D: diagonal -2(dx+dy), off-diagonal dy."""
    A = np.diag(np.full(n, -2.0 * (dx + dy)))
    A += np.diag(np.full(n - 1, dy), 1) + np.diag(np.full(n - 1, dy), -1)
    return A


def line_eigenvalues(n: int, dx: float, dy: float) -> np.ndarray:
    """Closed-form eigenvalues lambda_k, k = 1..n."""
    k = np.arange(1, n + 1, dtype=np.float64)
    return -2.0 * (dx + dy) + 2.0 * dy * np.cos(k * np.pi / (n + 1))


def mode_diagonal(n_modes: int, h: float, kappa: float) -> np.ndarray:
    """Diagonal of the per-mode tridiagonal system for uniform spacing h and the
    Helmholtz shift kappa: lambda_k + kappa with dx = dy = 1/h^2."""
    d = 1.0 / (h * h)
    return line_eigenvalues(n_modes, d, d) + kappa


# --------------------------------------------------------------------------- tridiagonal

def tridiag_solve_modes(F: np.ndarray, diag: np.ndarray, off: float) -> np.ndarray:
    """Solve tridiag(off, diag[k], off) y[:, k] = F[:, k] for every column k
    (rows are the tridiagonal direction).  LAPACK banded LU per mode."""
    F = np.asarray(F, dtype=np.float64)
    m, K = F.shape
    Y = np.empty_like(F)
    for k in range(K):
        ab = np.zeros((3, m))
        ab[0, 1:] = off
        ab[1, :] = diag[k]
        ab[2, :-1] = off
        Y[:, k] = scipy.linalg.solve_banded((1, 1), ab, F[:, k])
    return Y


def tridiag_dense(m: int, diag: float, off: float) -> np.ndarray:
    return (np.diag(np.full(m, diag)) + np.diag(np.full(m - 1, off), 1)
            + np.diag(np.full(m - 1, off), -1))


# --------------------------------------------------------------------------- rectangle operator

def rect_matrix(rows: int, cols: int, h: float, kappa: float) -> sp.csr_matrix:
    """5-point operator on a rows x cols block of unknowns with zero Dirichlet
    data all around; unknowns in row-major order (column index fastest)."""
    d = 1.0 / (h * h)
    Tc = sp.diags([np.full(cols - 1, d), np.full(cols, -2.0 * d), np.full(cols - 1, d)], [-1, 0, 1])
    Tr = sp.diags([np.full(rows - 1, d), np.full(rows, -2.0 * d), np.full(rows - 1, d)], [-1, 0, 1])
    A = sp.kron(sp.identity(rows), Tc) + sp.kron(Tr, sp.identity(cols)) + kappa * sp.identity(rows * cols)
    return A.tocsr()


def rect_solve(F: np.ndarray, h: float, kappa: float) -> np.ndarray:
    """Direct solve of the rectangle operator (SuperLU on the assembled matrix)."""
    F = np.asarray(F, dtype=np.float64)
    rows, cols = F.shape
    A = rect_matrix(rows, cols, h, kappa)
    import scipy.sparse.linalg as spla
    return spla.spsolve(A.tocsc(), F.ravel()).reshape(rows, cols)


def rect_apply(Z: np.ndarray, h: float, kappa: float) -> np.ndarray:
    rows, cols = Z.shape
    return (rect_matrix(rows, cols, h, kappa) @ np.asarray(Z, dtype=np.float64).ravel()).reshape(rows, cols)
