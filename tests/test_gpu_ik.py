"""The interface Krylov iteration (FDS_FLAG_INTERFACE_KRYLOV): the same
right-preconditioned GMRES(m) with its basis on the centre's interface lines.
Every solve is compared with the FP64 oracle (direct solution of the global
system) at the 1e-10 bar, and its iteration count with the full-vector
iteration's (equal iterates up to rounding)."""

import functools

import pytest

import workloads
from oracle import composite
from tests.gpu_util import compare, device_problem, log, oracle_solution

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _fds():
    import paper_2509_23180_amd as fds
    return fds


def _problem(shape, n, kappa, kind, seed=0):
    if kind == "manufactured":
        return workloads.manufactured_problem(shape, n, kappa)
    if kind == "shifted":
        return workloads.manufactured_problem(shape, n, kappa, shifted=True)
    return workloads.gaussian_problem(shape, n, kappa, 1, seed, 0)


def _ik_problem(prob, restart_m=30, max_cycles=200):
    import paper_2509_23180_amd as fds
    plan, rhs, bc, x = device_problem(prob, restart_m=restart_m, max_cycles=max_cycles)
    ik = fds.Plan(prob.rects, prob.h, prob.kappa, restart_m=restart_m, max_cycles=max_cycles,
                  flags=fds.FLAG_INTERFACE_KRYLOV)
    return ik, plan, rhs, bc, x


CASES = [
    ("cross", 32, 0.0, "manufactured"),
    ("cross", 32, 0.0, "shifted"),
    ("cross", 33, -50.0, "gauss"),
    ("L", 32, 0.0, "shifted"),
    ("L", 17, -100.0, "gauss"),
    ("T", 33, -50.0, "gauss"),
    ("T", 20, 0.0, "shifted"),
    ("pair", 20, -3.0, "shifted"),
    ("square", 17, 0.0, "shifted"),
    ("cross", 2, -1.0, "gauss"),
    ("cross", 3, 0.0, "shifted"),
    ("T", 7, 0.0, "gauss"),
    ("cross", 1, 0.0, "shifted"),          # centre of one node: the full-vector iteration
    ("cross", 100, -10.0, "gauss"),
]


@pytest.mark.parametrize("restart_m", [6, 30])
@pytest.mark.parametrize("shape,n,kappa,kind", CASES)
def test_ik_parity(shape, n, kappa, kind, restart_m):
    fds = _fds()
    prob = _problem(shape, n, kappa, kind)
    ref = oracle_solution(prob)
    ik, plan, rhs, bc, x = _ik_problem(prob, restart_m=restart_m)
    log(f"ik {shape} n={n} kappa={kappa} {kind} m={restart_m}")
    r_ik = fds.solve(ik, rhs, x, 1e-12, bc=bc)
    err = compare(prob, x, ref)
    log(f"  ik: its={r_ik.iterations} cycles={r_ik.cycles} stop={r_ik.stop_reason} err={err:.3e} "
        f"relres={r_ik.relres_schur:.2e} global={r_ik.relres_global:.2e}")
    assert r_ik.status == 0, r_ik
    assert err <= 1e-10
    assert r_ik.relres_global <= 1e-11
    x2 = torch.full_like(x, float("nan"))
    r_full = fds.solve(plan, rhs, x2, 1e-12, bc=bc)
    log(f"  full-vector: its={r_full.iterations} cycles={r_full.cycles}")
    assert abs(r_ik.iterations - r_full.iterations) <= max(2, r_full.iterations // 20)


@functools.lru_cache(maxsize=None)
def _large(shape, n, kappa, kind, seed):
    prob = _problem(shape, n, kappa, kind, seed)
    return prob, composite.solve(prob.rects, prob.h, prob.kappa, prob.f_grid, prob.g_grid, method="splu")


@pytest.mark.parametrize("shape,n,kappa,kind,seed", [("cross", 400, 0.0, "shifted", 0),
                                                     ("L", 512, -30.0, "gauss", 4),
                                                     ("T", 384, -75.0, "gauss", 2)])
def test_ik_large_parity(shape, n, kappa, kind, seed):
    """Sizes with several cross-sum tiles per line (384..512 nodes)."""
    fds = _fds()
    prob, ref = _large(shape, n, kappa, kind, seed)
    ik, plan, rhs, bc, x = _ik_problem(prob)
    log(f"ik large {shape} n={n}")
    r = fds.solve(ik, rhs, x, 1e-12, bc=bc)
    err = compare(prob, x, ref)
    log(f"  its={r.iterations} cycles={r.cycles} stop={r.stop_reason} err={err:.3e}")
    assert r.status == 0, r
    assert err <= 1e-10


@pytest.mark.parametrize("restart_m,shape,n,kappa,kind,seed", [(80, "cross", 400, 0.0, "shifted", 0),
                                                               (120, "L", 512, -30.0, "gauss", 4),
                                                               (80, "T", 450, 0.0, "gauss", 2)])
def test_ik_long_restart_parity(restart_m, shape, n, kappa, kind, seed):
    """Restart lengths 80 (the serving path's) and 120 (the most a plan
    takes): more than 64 steps in one cycle, which the MGS recurrence runs
    with two rows per lane; each case is checked against a solve whose
    first cycle runs past step 64."""
    fds = _fds()
    prob, ref = _large(shape, n, kappa, kind, seed)
    ik, plan, rhs, bc, x = _ik_problem(prob, restart_m=restart_m)
    log(f"ik {shape} n={n} m={restart_m}")
    r = fds.solve(ik, rhs, x, 1e-12, bc=bc)
    err = compare(prob, x, ref)
    log(f"  its={r.iterations} cycles={r.cycles} stop={r.stop_reason} err={err:.3e}")
    assert r.status == 0, r
    assert min(r.iterations, restart_m) > 64, r
    assert err <= 1e-10


def test_ik_long_lines_parity():
    """Lines of 1100 nodes: three source chunks and five target tiles in the
    cross-axis sums (L shape keeps the oracle in seconds)."""
    fds = _fds()
    prob = _problem("L", 1100, -20.0, "gauss", 5)
    ref = composite.solve(prob.rects, prob.h, prob.kappa, prob.f_grid, prob.g_grid, method="splu")
    ik, plan, rhs, bc, x = _ik_problem(prob, restart_m=40)
    r = fds.solve(ik, rhs, x, 1e-12, bc=bc)
    err = compare(prob, x, ref)
    log(f"ik L n=1100: its={r.iterations} cycles={r.cycles} stop={r.stop_reason} err={err:.3e}")
    assert r.status == 0, r
    assert err <= 1e-10


@pytest.mark.parametrize("graph", ["1", "0"])
def test_ik_batch_matches_standalone(graph, monkeypatch):
    """Each problem of a mixed batch gives bitwise the result of its solve
    alone (with captured cycles and kernel by kernel), and the oracle's."""
    fds = _fds()
    monkeypatch.setenv("FDS_GRAPH", graph)
    specs = [("cross", 24, 0.0, "gauss", 0), ("L", 40, -70.0, "gauss", 1), ("T", 9, -5.0, "shifted", 0),
             ("cross", 64, -20.0, "gauss", 2), ("square", 30, 0.0, "gauss", 3), ("T", 130, -1.0, "gauss", 4)]
    probs = [_problem(s, n, k, kind, seed) for (s, n, k, kind, seed) in specs]
    alone = []
    items = []
    for p in probs:
        ik, plan, rhs, bc, x = _ik_problem(p, restart_m=8)
        r = fds.solve(ik, rhs, x, 1e-12, bc=bc)
        assert r.status == 0, r
        alone.append((x.clone(), r))
        items.append((ik, rhs, bc, torch.full_like(x, float("nan"))))
    res = fds.solve_batch([i[0] for i in items], [i[1] for i in items], [i[3] for i in items],
                          [1e-12] * len(items), bcs=[i[2] for i in items])
    for (x_alone, r_alone), it, r, p in zip(alone, items, res, probs):
        assert r.status == 0
        assert r.iterations == r_alone.iterations
        assert torch.equal(it[3], x_alone)
        err = compare(p, it[3], oracle_solution(p))
        log(f"ik batch {p.shape} n={p.n}: its={r.iterations} err={err:.3e}")
        assert err <= 1e-10


def test_ik_server_mix_matches_oracle():
    """Interface-iteration requests served next to full-vector ones."""
    import time
    fds = _fds()
    probs = [_problem("cross", 48, 0.0, "gauss", 1), _problem("T", 40, -20.0, "gauss", 2),
             _problem("L", 33, -10.0, "gauss", 5)]
    srv = fds.Server(hbm_budget_bytes=1 << 30, max_slots=8)
    items, tickets = [], []
    for k, p in enumerate(probs):
        ik, plan, rhs, bc, x = _ik_problem(p)
        use = ik if k != 1 else plan
        items.append((use, rhs, bc, x))
        tickets.append(srv.submit(use, rhs, x, 1e-11, bc=bc))
    results = {}
    t0 = time.time()
    while len(results) < len(tickets) and time.time() - t0 < 60:
        for t in tickets:
            if t not in results:
                r = srv.poll(t)
                if r is not None:
                    results[t] = r
        time.sleep(0.001)
    srv.close()
    assert len(results) == len(tickets)
    for p, it, t in zip(probs, items, tickets):
        assert results[t].status == 0
        assert compare(p, it[3], oracle_solution(p)) <= 1e-10


def test_ik_flag_needs_fp64():
    fds = _fds()
    rects = workloads.shape_rects("cross", 8)
    with pytest.raises(fds.FdsError) as ei:
        fds.Plan(rects, 1.0 / 9, 0.0, precision=fds.FP32_PRECOND, flags=fds.FLAG_INTERFACE_KRYLOV)
    assert ei.value.status == -1
    with pytest.raises(fds.FdsError):
        fds.Plan(rects, 1.0 / 9, 0.0, flags=4)
