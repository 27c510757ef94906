"""Pins of the Schur-complement oracle and the reference GMRES."""

import numpy as np
import pytest

from oracle import composite, rect, schur
import workloads


def _op(shape, n, kappa=0.0, seed=0):
    prob = workloads.gaussian_problem(shape, n, kappa, 7, seed, 0)
    P = schur.partition(prob.rects, prob.h, prob.kappa, prob.f_grid, prob.g_grid)
    return prob, P, schur.SchurOperator(P)


@pytest.mark.parametrize("shape", ["cross", "L", "T", "pair"])
def test_block_elimination_reproduces_global_solution(shape):
    """Schur equations + back substitution (Section 2.3, Algorithm 1) give
    exactly the global solution."""
    prob, P, op = _op(shape, 6, -20.0)
    glob = composite.solve(prob.rects, prob.h, prob.kappa, prob.f_grid, prob.g_grid, method="dense")
    Lc = op.dense_L()
    pc = np.linalg.solve(Lc, op.fprime())
    assert np.allclose(pc, glob.p[P.centre], rtol=1e-12, atol=1e-12 * abs(glob.p).max())
    pr = op.back_substitute(pc)
    assert np.allclose(pr, glob.p[P.rest], rtol=1e-12, atol=1e-12 * abs(glob.p).max())


@pytest.mark.parametrize("shape", ["cross", "L", "T"])
def test_schur_operator_symmetric_negative_definite(shape):
    _, _, op = _op(shape, 6)
    L = op.dense_L()
    assert np.abs(L - L.T).max() < 1e-12 * np.abs(L).max()
    assert np.linalg.eigvalsh(0.5 * (L + L.T)).max() < 0.0


@pytest.mark.parametrize("shape", ["cross", "L", "T"])
def test_preconditioned_spectrum(shape):
    """A_c^{-1} S has real eigenvalues in [0, 1), so I - A_c^{-1} S (the
    preconditioned operator) has spectrum in (0, 1]."""
    _, _, op = _op(shape, 6)
    n = op.Acc.shape[0]
    M = np.column_stack([op.apply_Minv(c) for c in op.dense_S().T])
    ev = np.linalg.eigvals(M)
    assert np.abs(ev.imag).max() < 1e-10
    assert ev.real.min() > -1e-12 and ev.real.max() < 1.0


def test_krylov_dimension_bounded_by_interface():
    """S is supported on the centre's boundary lines, so the preconditioned
    Krylov space has dimension at most |Gamma| + 1 (|Gamma| = 4n-4 for the cross)."""
    n = 5
    _, _, op = _op("cross", n)
    L = op.dense_L()
    Minv = np.linalg.inv(op.Acc.toarray())
    B = L @ Minv
    v = op.fprime()
    K = [v / np.linalg.norm(v)]
    for _ in range(4 * n + 4):
        w = B @ K[-1]
        K.append(w / np.linalg.norm(w))
    rank = np.linalg.matrix_rank(np.array(K), tol=1e-9)
    assert rank <= (4 * n - 4) + 1


@pytest.mark.parametrize("kappa", [0.0, -50.0])
@pytest.mark.parametrize("shape", ["cross", "L"])
def test_arm_schur_block_is_diagonal_in_sine_basis(shape, kappa):
    """S_ca = delta^2 Q diag(g) Q on the centre line next to arm a, with
    g_k = -sinh(m t_k)/(delta sinh((m+1) t_k)), cosh t_k = -a_k/(2 delta),
    a_k = -4 delta + 2 delta cos(k pi/(n+1)) + kappa, m = n+1 arm rows."""
    n = 7
    prob, P, op = _op(shape, n, kappa)
    d = 1.0 / prob.h ** 2
    k = np.arange(1, n + 1)
    a = -4 * d + 2 * d * np.cos(k * np.pi / (n + 1)) + kappa
    t = np.arccosh(-a / (2 * d))
    m = n + 1
    g = -np.sinh(m * t) / (d * np.sinh((m + 1) * t))
    Q = rect.sine_eigvecs(n)
    line = d * d * Q @ np.diag(g) @ Q
    for arm in range(len(P.arms)):
        S = schur.arm_schur_block(P, arm)
        nz = np.nonzero(np.abs(S).sum(axis=1))[0]
        assert len(nz) == n
        blk = S[np.ix_(nz, nz)]
        assert np.abs(blk - line).max() < 1e-12 * np.abs(line).max()


def test_mgs_and_givens():
    rng = np.random.default_rng(3)
    V = np.linalg.qr(rng.normal(size=(50, 4)))[0].T
    w = rng.normal(size=50)
    h, v = schur.mgs_step(V, w)
    assert np.abs(V @ v).max() < 1e-14
    assert abs(np.linalg.norm(v) - 1) < 1e-14
    assert np.allclose(V.T @ h[:4] + h[4] * v, w, atol=1e-13)
    c, s, rho = schur.givens(3.0, 4.0)
    assert (c, s, rho) == (0.6, 0.8, 5.0)
    assert c * 3 + s * 4 == pytest.approx(rho, rel=1e-15)
    assert abs(-s * 3 + c * 4) < 1e-15


@pytest.mark.parametrize("shape", ["cross", "T"])
def test_reference_gmres_converges_to_direct_solution(shape):
    prob, P, op = _op(shape, 12, -5.0)
    glob = composite.solve(prob.rects, prob.h, prob.kappa, prob.f_grid, prob.g_grid)
    res = schur.gmres_right(op.apply_L, op.apply_Minv, op.fprime(), m=10, tol=1e-12)
    assert res.converged
    ref = glob.p[P.centre]
    assert np.abs(res.x - ref).max() <= 1e-10 * np.abs(ref).max()
    # the Givens residual estimate tracks the true residual
    true = np.linalg.norm(op.fprime() - op.apply_L(res.x)) / np.linalg.norm(op.fprime())
    assert true <= 1e-11


def test_preconditioner_cuts_iterations():
    """Section 3.2: the A_c^{-1} preconditioner needs far fewer iterations
    than no preconditioner."""
    prob, P, op = _op("cross", 16)
    f = op.fprime()
    pre = schur.gmres_right(op.apply_L, op.apply_Minv, f, m=40, tol=1e-8, max_cycles=50)
    nop = schur.gmres_right(op.apply_L, lambda v: np.array(v), f, m=40, tol=1e-8, max_cycles=50)
    assert pre.converged
    assert nop.iterations > 5 * pre.iterations


def _corner_inverse(m, delta, a):
    """[T^-1]_11 of the m x m tridiagonal (delta, a, delta), by a dense inverse."""
    T = np.diag(np.full(m, a)) + delta * (np.eye(m, k=1) + np.eye(m, k=-1))
    return np.linalg.inv(T)[0, 0]


ARMS = {"cross": ("S", "N", "W", "E"), "L": ("N", "E"), "T": ("W", "E", "S")}


@pytest.mark.parametrize("shape", ["cross", "L", "T"])
@pytest.mark.parametrize("kappa", [0.0, -30.0])
def test_jacobi_diagonal_closed_form(shape, kappa):
    """diag(L_c) (Section 3.2's Jacobi preconditioner) from the assembled
    blocks equals its closed form: -4 delta + kappa, minus on each boundary
    line next to an arm delta^2 sum_k (2/N) sin^2(pi i k/N) [T_k^-1]_11, where
    T_k = tridiag(delta, 2 delta (cos(k pi/N) - 2) + kappa, delta) is the arm's
    mode-k system over its n+1 rows (Section 2.1's per-mode decomposition);
    corners take both lines' terms."""
    n = 7
    _, P, op = _op(shape, n, kappa)
    h = 1.0 / (n + 1)
    delta = 1.0 / h ** 2
    N = n + 1
    want = np.full((n, n), -4 * delta + kappa)
    i = np.arange(1, n + 1)
    line = np.zeros(n)
    for k in range(1, n + 1):
        g = _corner_inverse(n + 1, delta, 2 * delta * (np.cos(k * np.pi / N) - 2) + kappa)
        line += delta ** 2 * (2.0 / N) * np.sin(np.pi * i * k / N) ** 2 * g
    for arm in ARMS[shape]:
        if arm == "S":
            want[0, :] -= line
        elif arm == "N":
            want[-1, :] -= line
        elif arm == "W":
            want[:, 0] -= line
        else:
            want[:, -1] -= line
    got = op.jacobi_diagonal().reshape(n, n)
    assert np.abs(got - want).max() <= 1e-12 * delta


def test_jacobi_preconditioned_gmres_reaches_solution_slowly():
    """GMRES preconditioned by the Jacobi diagonal reaches the direct solution
    of the interface system, with several times the iterations of the A_c^-1
    preconditioner (Section 3.2, Fig. 4)."""
    prob, P, op = _op("cross", 12, 0.0)
    f = op.fprime()
    ref = np.linalg.solve(op.dense_L(), f)
    jac = schur.gmres_right(op.apply_L, op.apply_Jinv, f, m=30, tol=1e-11, max_cycles=100)
    pre = schur.gmres_right(op.apply_L, op.apply_Minv, f, m=30, tol=1e-11, max_cycles=100)
    assert jac.converged and pre.converged
    assert np.abs(jac.x - ref).max() <= 1e-9 * np.abs(ref).max()
    assert jac.iterations >= 3 * pre.iterations, (jac.iterations, pre.iterations)
