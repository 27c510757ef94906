"""Whole-solve parity with the FP64 oracle at the sizes the benchmark
configurations run: centres of more than 64 Gram blocks (the two-level block
reduction of the Gram passes), both the plain FP64 GMRES(30) and the
FP32-preconditioned flexible GMRES(40), against the sparse direct solution of
the global system; and mixed batches of uneven sizes against the oracle."""

import functools

import numpy as np
import pytest

import workloads
from oracle import composite
from tests.gpu_util import compare, device_problem, log

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _fds():
    import paper_2509_23180_amd as fds
    return fds


def _problem(shape, n, kappa, kind, seed):
    if kind == "shifted":
        return workloads.manufactured_problem(shape, n, kappa, shifted=True)
    return workloads.gaussian_problem(shape, n, kappa, 1, seed, 0)


@functools.lru_cache(maxsize=None)
def _oracle(shape, n, kappa, kind, seed):
    prob = _problem(shape, n, kappa, kind, seed)
    log(f"oracle {shape} n={n} kappa={kappa} {kind} (SuperLU)")
    return prob, composite.solve(prob.rects, prob.h, prob.kappa, prob.f_grid, prob.g_grid, method="splu")


# n = 400 and 512: 79 and 128 Gram blocks per problem (more than 64)
LARGE = [("cross", 400, 0.0, "shifted", 0), ("L", 512, -30.0, "gauss", 4), ("T", 384, -75.0, "gauss", 2)]


@pytest.mark.parametrize("precision,restart_m", [(0, 30), (1, 40)])
@pytest.mark.parametrize("shape,n,kappa,kind,seed", LARGE)
def test_large_parity(shape, n, kappa, kind, seed, precision, restart_m):
    fds = _fds()
    prob, ref = _oracle(shape, n, kappa, kind, seed)
    log(f"solve {shape} n={n} kappa={kappa} {kind} precision={precision} m={restart_m}")
    plan, rhs, bc, x = device_problem(prob, restart_m=restart_m, precision=precision)
    res = fds.solve(plan, rhs, x, 1e-12, bc=bc)
    err = compare(prob, x, ref)
    log(f"  its={res.iterations} cycles={res.cycles} stop={res.stop_reason} err={err:.3e} "
        f"relres={res.relres_schur:.2e} global={res.relres_global:.2e}")
    assert res.status == 0, res
    assert err <= 1e-10


def test_large_mixed_batch_against_oracle():
    """A batch of uneven sizes (two-level and single-level Gram reductions in
    the same launches), FP32-preconditioned FGMRES(40), each against the
    oracle at the FP64 bar."""
    fds = _fds()
    specs = [("L", 512, -30.0, "gauss", 4), ("cross", 64, -10.0, "gauss", 1), ("T", 128, 0.0, "gauss", 5),
             ("cross", 400, 0.0, "shifted", 0)]
    pairs = [_oracle(*s) for s in specs]
    items = [device_problem(p, restart_m=40, precision=1) for p, _ in pairs]
    log("batch of 4 (n = 512, 64, 128, 400), FGMRES(40)")
    res = fds.solve_batch([i[0] for i in items], [i[1] for i in items], [i[3] for i in items],
                          [1e-12] * len(items), bcs=[i[2] for i in items])
    for (prob, ref), it, r in zip(pairs, items, res):
        err = compare(prob, it[3], ref)
        log(f"  {prob.shape} n={prob.n}: its={r.iterations} err={err:.3e}")
        assert r.status == 0, r
        assert err <= 1e-10


def test_restart_length_120():
    """The longest restart the plan accepts.  Without preconditioner (P = I)
    the first cycle runs all 120 Arnoldi steps (the Gram step's LDS then
    exceeds 64 KiB and is opted in per kernel); with A_c^-1 both variants
    converge within the first cycle.  Every solve reaches the oracle."""
    fds = _fds()
    prob = workloads.gaussian_problem("cross", 48, -5.0, 1, 9, 0)
    ref = composite.solve(prob.rects, prob.h, prob.kappa, prob.f_grid, prob.g_grid)
    for precision in (2, 0, 1):
        plan, rhs, bc, x = device_problem(prob, restart_m=120, precision=precision, max_cycles=100)
        res = fds.solve(plan, rhs, x, 1e-12, bc=bc)
        err = compare(prob, x, ref)
        log(f"restart 120 precision={precision}: its={res.iterations} cycles={res.cycles} "
            f"stop={res.stop_reason} err={err:.3e}")
        assert res.status == 0, res
        if precision == 2:
            assert res.cycles >= 2 and res.iterations > 120, res
        assert err <= 1e-10
