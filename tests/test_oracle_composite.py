"""Pins of the global composite oracle against hand-derived fixtures, exact
polynomial solutions, closed-form counts and the discretisation order."""

import json
import os

import numpy as np
import pytest

from oracle import composite, layout, rect
import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _const_grid(n, value):
    N = n + 1
    return np.full((3 * N + 1, 3 * N + 1), float(value))


@pytest.mark.parametrize("fname", ["cross_n1.json", "L_n1.json"])
def test_golden_hand_derived(fname):
    with open(os.path.join(GOLDEN, fname)) as fh:
        gd = json.load(fh)
    n = gd["n"]
    rects = workloads.shape_rects(gd["shape"], n)
    h = 1.0 / (n + 1)
    sol = composite.solve(rects, h, gd["kappa"], _const_grid(n, gd["f"]), _const_grid(n, gd["g"]),
                          method="dense")
    P = sol.on_grid()
    vals = gd["values"]
    i, j = vals["centre"]["node"]
    assert P[j, i] == pytest.approx(vals["centre"]["num"] / vals["centre"]["den"], rel=1e-14)
    for key in ("interface", "arm"):
        for i, j in vals[key]["nodes"]:
            assert P[j, i] == pytest.approx(vals[key]["num"] / vals[key]["den"], rel=1e-14)
    assert sol.grid.n_unknowns == 1 + 2 * len(vals["interface"]["nodes"])


@pytest.mark.parametrize("shape,count", [("cross", lambda n: 5 * n * n + 4 * n),
                                         ("L", lambda n: 3 * n * n + 2 * n),
                                         ("T", lambda n: 4 * n * n + 3 * n)])
@pytest.mark.parametrize("n", [1, 2, 5, 32])
def test_unknown_counts(shape, count, n):
    g = composite.classify(workloads.shape_rects(shape, n))
    assert g.n_unknowns == count(n)


def _cubic(x, y):
    return x ** 3 + 2.0 * y ** 3 - x * y * y + 3.0 * x - 1.0 + 0.5 * x * x * y


def _cubic_lap(x, y):
    # d2/dx2: 6x + y ; d2/dy2: 12y - 2x
    return 6.0 * x + y + 12.0 * y - 2.0 * x


@pytest.mark.parametrize("shape", ["cross", "L", "T", "square", "pair"])
@pytest.mark.parametrize("kappa", [0.0, -50.0, 7.5])
def test_cubic_polynomials_are_exact(shape, kappa):
    """The five-point Laplacian is exact on polynomials of degree <= 3, so the
    discrete solution with f = lap(p) + kappa p and Dirichlet data p equals p at
    every unknown (exercises delta, signs, kappa, the boundary lift, interface
    ownership and reentrant corners)."""
    n = 6
    X, Y, h = workloads.frame_nodes(n)
    p = _cubic(X, Y)
    f = _cubic_lap(X, Y) + kappa * p
    rects = workloads.shape_rects(shape, n)
    sol = composite.solve(rects, h, kappa, f, p, method="band_lu")
    P = sol.on_grid()
    m = sol.grid.unknown
    p = p[:P.shape[0], :P.shape[1]]
    assert np.max(np.abs(P[m] - p[m])) <= 1e-11 * np.max(np.abs(p[m]))


@pytest.mark.parametrize("shape", ["cross", "L", "T"])
def test_band_solvers_agree_with_dense(shape):
    n = 7
    prob = workloads.gaussian_problem(shape, n, -13.0, 99, 0, 0)
    ref = composite.solve(prob.rects, prob.h, prob.kappa, prob.f_grid, prob.g_grid, method="dense")
    for meth in ("band", "band_lu", "splu"):
        s = composite.solve(prob.rects, prob.h, prob.kappa, prob.f_grid, prob.g_grid, method=meth)
        assert np.max(np.abs(s.p - ref.p)) <= 1e-13 * np.max(np.abs(ref.p))
        assert s.relres < 1e-13


@pytest.mark.parametrize("method", ["band", "splu"])
def test_solve_many_matches_dense_per_rhs(method):
    """One factorisation for several right-hand sides gives each dense solve."""
    probs = [workloads.gaussian_problem("T", 6, -4.0, 98, 0, r) for r in range(3)]
    probs.append(workloads.manufactured_problem("T", 6, -4.0, shifted=True))
    p0 = probs[0]
    sols = composite.solve_many(p0.rects, p0.h, p0.kappa, [(q.f_grid, q.g_grid) for q in probs],
                                method=method)
    for q, s in zip(probs, sols):
        ref = composite.solve(q.rects, q.h, q.kappa, q.f_grid, q.g_grid, method="dense")
        assert np.max(np.abs(s.p - ref.p)) <= 1e-13 * np.max(np.abs(ref.p))
        assert s.relres < 1e-13


def test_matrix_symmetric():
    """R_ij = R_ji^T for the self-adjoint operator (Section 2.3)."""
    prob = workloads.manufactured_problem("T", 9, -3.0)
    A, _, _ = composite.assemble(prob.rects, prob.h, prob.kappa, prob.f_grid, prob.g_grid)
    assert abs(A - A.T).max() == 0.0


def test_second_order_convergence():
    """Manufactured solution on the cross: max error falls 4x per halving of h
    (Section 3.1 reports second order)."""
    errs = []
    for N in (16, 32, 64, 128):
        prob = workloads.manufactured_problem("cross", N - 1, 0.0, shifted=True)
        sol = composite.solve(prob.rects, prob.h, 0.0, prob.f_grid, prob.g_grid)
        P = sol.on_grid()
        m = sol.grid.unknown
        errs.append(np.max(np.abs(P[m] - prob.p_exact[m])))
    ratios = [errs[k] / errs[k + 1] for k in range(3)]
    for r in ratios:
        assert 3.7 < r < 4.3, ratios


def test_coupling_matters():
    """Solving the five squares separately (interfaces forced to the exact
    boundary value zero) differs from the coupled solve; a dropped coupling in
    the assembly would make them equal."""
    n = 32
    prob = workloads.gaussian_problem("cross", n, 0.0, 1, 0, 0)
    sol = composite.solve(prob.rects, prob.h, 0.0, prob.f_grid, prob.g_grid)
    P = sol.on_grid()
    # decoupled: every square on its own with zero data on its whole boundary
    D = np.zeros_like(P)
    for (i0, j0, i1, j1) in prob.rects:
        F = prob.f_grid[j0 + 1:j1, i0 + 1:i1]
        D[j0 + 1:j1, i0 + 1:i1] = rect.rect_solve(F, prob.h, 0.0)
    m = sol.grid.unknown
    diff = np.max(np.abs(P[m] - D[m])) / np.max(np.abs(P[m]))
    assert diff > 1e-3


def test_layout_roundtrip_and_sizes():
    for shape in ("cross", "L", "T"):
        n = 5
        rects = workloads.shape_rects(shape, n)
        g = composite.classify(rects)
        own = layout.owned_nodes(rects)
        total = sum(len(jj) for jj, _ in own)
        assert total == g.n_unknowns
        seen = np.zeros_like(g.unknown)
        for jj, ii in own:
            assert g.unknown[jj, ii].all()
            assert not seen[jj, ii].any()
            seen[jj, ii] = True
        assert (seen == g.unknown).all()
        shapes = layout.block_shapes(rects)
        assert shapes[0] == (n, n)
        assert sorted(shapes[1:]) == sorted([(n, n + 1) if (r[2] - r[0]) == (n + 1) and
                                             (r[0] == rects[0][2] or r[2] == rects[0][0])
                                             else (n + 1, n) for r in rects[1:]])
        vals = np.random.default_rng(0).normal(size=g.unknown.shape)
        back = layout.from_user(rects, layout.to_user(rects, vals), vals.shape)
        assert np.array_equal(back[g.unknown], vals[g.unknown])


# ---------------------------------------------------------------------------
# Chains of rectangles: several coupled subdomains (closing remark of
# Section 2.4: the method carries over to longer concatenations)
# ---------------------------------------------------------------------------

CHAINS = [
    (6, [7, 7, 7, 7], True),          # four squares stacked
    (5, [4, 9, 3, 6, 5], False),      # five rectangles of unequal length in a row
    (4, [5, 5, 5], True),             # three: one coupled rectangle (the L/T case)
]


@pytest.mark.parametrize("n,lengths,vertical", CHAINS)
@pytest.mark.parametrize("kappa", [0.0, -30.0])
def test_cubic_polynomials_are_exact_on_chains(n, lengths, vertical, kappa):
    rects = workloads.chain_rects(n, lengths, vertical)
    h = 1.0 / (n + 1)
    I = max(r[2] for r in rects)
    J = max(r[3] for r in rects)
    X, Y = np.meshgrid(np.arange(I + 1) * h, np.arange(J + 1) * h, indexing="xy")
    p = _cubic(X, Y)
    sol = composite.solve(rects, h, kappa, _cubic_lap(X, Y) + kappa * p, p, method="band_lu")
    P = sol.on_grid()
    m = sol.grid.unknown
    assert m.sum() == sum((r[2] - r[0] - 1) * (r[3] - r[1] - 1) for r in rects) + (len(rects) - 1) * n
    assert np.max(np.abs(P[m] - p[m])) <= 1e-11 * np.max(np.abs(p[m]))


@pytest.mark.parametrize("n,lengths,vertical", CHAINS)
@pytest.mark.parametrize("order", ["chain", "reversed", "shuffled"])
def test_chain_layout_owns_every_unknown_once(n, lengths, vertical, order):
    rects = workloads.chain_rects(n, lengths, vertical)
    if order == "reversed":
        rects = rects[::-1]
    elif order == "shuffled":
        rects = [rects[k] for k in np.random.default_rng(len(rects)).permutation(len(rects))]
    g = composite.classify(rects)
    own = layout.owned_nodes(rects)
    seen = np.zeros(g.unknown.shape, dtype=int)
    for jj, ii in own:
        seen[jj, ii] += 1
    assert (seen[g.unknown] == 1).all() and (seen[~g.unknown] == 0).all()
    # the ends are the non-coupled rectangles; each owns the line it shares
    coupled = layout.coupled_indices(rects)
    assert len(coupled) == len(rects) - 2
    for r, (jj, ii) in enumerate(own):
        i0, j0, i1, j1 = rects[r]
        if r not in coupled:
            assert len(jj) == (i1 - i0 - 1) * (j1 - j0 - 1) + n
    # a line between two coupled rectangles goes to the one listed first
    for r in coupled:
        for q in coupled:
            a, b = rects[r], rects[q]
            if r < q and (a[3] == b[1] or a[1] == b[3] or a[2] == b[0] or a[0] == b[2]) and \
                    ((a[0], a[2]) == (b[0], b[2]) or (a[1], a[3]) == (b[1], b[3])):
                jj, ii = own[r]
                if vertical:
                    line_j = a[3] if a[3] == b[1] else a[1]
                    assert (jj == line_j).sum() == n
                else:
                    line_i = a[2] if a[2] == b[0] else a[0]
                    assert (ii == line_i).sum() == n


@pytest.mark.parametrize("rects", [
    workloads.chain_rects(5, [6, 6, 6, 6], True),
    workloads.chain_rects(4, [5, 8, 3, 5, 7], False)[::-1],
    workloads.shape_rects("cross", 5), workloads.shape_rects("T", 4), workloads.shape_rects("pair", 3),
])
def test_product_layout_helper_matches_oracle_layout(rects):
    """The package's packing helper cuts the same owned blocks as the
    oracle's layout (two independent statements of the header's rule)."""
    from paper_2509_23180_amd import layout as plog
    own = layout.owned_nodes(rects)
    for r in range(len(rects)):
        ilo, ihi, jlo, jhi = plog.owned_box(rects, r)
        jj, ii = own[r]
        assert (jj.min(), jj.max(), ii.min(), ii.max()) == (jlo, jhi, ilo, ihi)
        assert len(jj) == (jhi - jlo + 1) * (ihi - ilo + 1)
