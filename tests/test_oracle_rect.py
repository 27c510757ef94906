"""Pins of the single-rectangle oracle pieces: sine transform, closed-form
eigenvalues, tridiagonal mode solves and the rectangle operator."""

import numpy as np
import pytest
import scipy.fft

from oracle import composite, rect


@pytest.mark.parametrize("n", [1, 2, 7, 32, 64, 100])
def test_dst_matches_library(n):
    """scipy's type-1 DST is 2*sum x_j sin(pi (j)(k)/(n+1)) (1-based)."""
    x = np.random.default_rng(n).normal(size=(3, n))
    ref = scipy.fft.dst(x, type=1, axis=-1) / 2.0
    assert np.allclose(rect.dst1_rows(x), ref, rtol=0, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("n", [1, 5, 32, 33, 256])
def test_dst_involution(n):
    S = rect.dst1_matrix(n)
    assert np.abs(S @ S - (n + 1) / 2.0 * np.eye(n)).max() < 1e-12 * n


@pytest.mark.parametrize("n", [8, 31])
def test_dst_of_sine_mode_is_delta(n):
    k0 = 3
    j = np.arange(1, n + 1)
    x = np.sin(np.pi * j * k0 / (n + 1))
    X = rect.dst1_rows(x[None, :])[0]
    e = np.zeros(n)
    e[k0 - 1] = (n + 1) / 2.0
    assert np.abs(X - e).max() < 1e-12 * n


@pytest.mark.parametrize("n,dx,dy", [(6, 4.0, 9.0), (20, 1.0, 1.0), (33, 1089.0, 1089.0)])
def test_line_eigen_decomposition(n, dx, dy):
    """Lambda = Q A Q^T with the closed-form eigenvalues (Section 2.1)."""
    A = rect.line_matrix(n, dx, dy)
    Q = rect.sine_eigvecs(n)
    lam = rect.line_eigenvalues(n, dx, dy)
    assert np.allclose(np.sort(np.linalg.eigvalsh(A)), np.sort(lam), atol=1e-10 * abs(lam).max())
    assert np.abs(Q @ A @ Q.T - np.diag(lam)).max() < 1e-10 * abs(lam).max()
    assert np.abs(Q @ Q.T - np.eye(n)).max() < 1e-13


def test_tridiag_modes_match_dense():
    rng = np.random.default_rng(1)
    m, K = 17, 9
    diag = -2.5 - rng.uniform(0, 3, size=K)
    F = rng.normal(size=(m, K))
    Y = rect.tridiag_solve_modes(F, diag, 1.0)
    for k in range(K):
        ref = np.linalg.solve(rect.tridiag_dense(m, diag[k], 1.0), F[:, k])
        assert np.allclose(Y[:, k], ref, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("m", [1, 2, 5, 40])
def test_tridiag_corner_closed_form(m):
    """For T = delta*tridiag(1, -2 cosh(t), 1) of size m the corner entry of the
    inverse is -sinh(m t)/(delta sinh((m+1) t)) (Chebyshev recurrence)."""
    delta, t = 3.0, 0.37
    T = rect.tridiag_dense(m, -2.0 * delta * np.cosh(t), delta)
    Ti = np.linalg.inv(T)
    closed = -np.sinh(m * t) / (delta * np.sinh((m + 1) * t))
    assert Ti[0, 0] == pytest.approx(closed, rel=1e-12)
    assert Ti[-1, -1] == pytest.approx(closed, rel=1e-12)


@pytest.mark.parametrize("rows,cols,a,b,kappa", [(9, 9, 1, 2, 0.0), (12, 7, 3, 1, -50.0),
                                                 (31, 31, 5, 4, -1.0)])
def test_rect_eigenfunction(rows, cols, a, b, kappa):
    """sin(a pi x) sin(b pi y) on a grid with x = c/(cols+1), y = r/(rows+1)
    (uniform h requires cols == rows for a square; here h is per-direction
    through the choice h = 1/(cols+1) = 1/(rows+1) only when equal, so the test
    uses the rectangle's own spacing along each axis via separate sines)."""
    h = 1.0 / (max(rows, cols) + 1)
    c = np.arange(1, cols + 1)
    r = np.arange(1, rows + 1)
    ux = np.sin(a * np.pi * c / (cols + 1))
    uy = np.sin(b * np.pi * r / (rows + 1))
    U = np.outer(uy, ux)
    d = 1.0 / (h * h)
    lam = d * (2 * np.cos(a * np.pi / (cols + 1)) - 2) + d * (2 * np.cos(b * np.pi / (rows + 1)) - 2) + kappa
    AU = rect.rect_apply(U, h, kappa)
    assert np.abs(AU - lam * U).max() < 1e-9 * abs(lam)
    Z = rect.rect_solve(U, h, kappa)
    assert np.abs(Z - U / lam).max() < 1e-12 * np.abs(U / lam).max()


def test_rect_matrix_matches_composite_single_square():
    """Two independently written assemblies agree on one square."""
    n = 6
    h = 1.0 / (n + 1)
    N = n + 1
    A, _, _ = composite.assemble([(0, 0, N, N)], h, -4.0, np.zeros((N + 1, N + 1)),
                                 np.zeros((N + 1, N + 1)))
    B = rect.rect_matrix(n, n, h, -4.0)
    assert abs(A - B).max() == 0.0


def test_dst_matrix_entries_exact_for_large_n():
    """Entries of the sine matrix agree with 50-digit arithmetic even where
    j*k is large (checks the exact reduction of the angle)."""
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 50
    n = 2047
    S = rect.dst1_matrix(n)
    rng = np.random.default_rng(0)
    for j, k in rng.integers(1, n + 1, size=(300, 2)):
        ref = float(mpmath.sin(mpmath.pi * int(j) * int(k) / (n + 1)))
        assert abs(S[j - 1, k - 1] - ref) <= 1e-15


@pytest.mark.parametrize("n,h,kappa", [(1, 0.5, 0.0), (6, 1.0 / 7, -50.0), (17, 1.0 / 18, 3.0),
                                       (40, 0.01, -100.0)])
def test_mode_diagonal_is_shifted_line_spectrum(n, h, kappa):
    """mode_diagonal is the spectrum of the x-direction line operator of the
    5-point scheme plus the y-direction centre weight and kappa (Section 2.1):
    eigenvalues of delta*tridiag(1, -2, 1) (built here from the stencil, not
    from the oracle), shifted by -2 delta + kappa, sorted alike."""
    d = 1.0 / (h * h)
    T = np.zeros((n, n))
    for i in range(n):
        T[i, i] = -2.0 * d
        if i > 0:
            T[i, i - 1] = d
        if i + 1 < n:
            T[i, i + 1] = d
    ref = np.sort(np.linalg.eigvalsh(T + (kappa - 2.0 * d) * np.eye(n)))
    got = np.sort(rect.mode_diagonal(n, h, kappa))
    assert np.abs(got - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("rows,cols,kappa", [(5, 4, 0.0), (3, 7, -30.0), (6, 6, 2.5)])
def test_mode_diagonal_block_diagonalises_rectangle(rows, cols, kappa):
    """Transforming the rectangle operator along x with the orthonormal sine
    basis (written out here) leaves, for every mode k, the tridiagonal system
    tridiag(delta, mode_diagonal[k], delta) along y: the per-mode systems the
    fast solver runs (Section 2.1)."""
    h = 1.0 / (max(rows, cols) + 1)
    d = 1.0 / (h * h)
    j = np.arange(1, cols + 1)
    Q = np.sqrt(2.0 / (cols + 1)) * np.sin(np.pi * np.outer(j, j) / (cols + 1))
    A = rect.rect_matrix(rows, cols, h, kappa).toarray()
    B = np.kron(np.eye(rows), Q) @ A @ np.kron(np.eye(rows), Q.T)
    diag = rect.mode_diagonal(cols, h, kappa)
    for k in range(cols):
        idx = np.arange(rows) * cols + k
        blk = B[np.ix_(idx, idx)]
        ref = np.diag(np.full(rows, diag[k])) + d * (np.eye(rows, k=1) + np.eye(rows, k=-1))
        assert np.abs(blk - ref).max() <= 1e-10 * d
        off = B[idx][:, np.setdiff1d(np.arange(rows * cols), idx)]
        assert np.abs(off).max() <= 1e-10 * d
