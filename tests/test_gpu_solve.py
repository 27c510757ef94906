"""Whole-solve parity with the FP64 oracle (global composite direct solve),
error paths, batching and serving."""

import numpy as np
import pytest

import workloads
from tests.gpu_util import compare, device_problem, log, oracle_solution

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _fds():
    import paper_2509_23180_amd as fds
    return fds


CASES_SMALL = [
    ("cross", 32, 0.0, "manufactured"),
    ("cross", 32, 0.0, "shifted"),
    ("cross", 32, -50.0, "gauss"),
    ("L", 32, 0.0, "shifted"),
    ("T", 33, -50.0, "gauss"),
    ("pair", 20, -3.0, "shifted"),
    ("square", 17, 0.0, "shifted"),
    ("cross", 1, 0.0, "shifted"),
    ("cross", 2, -1.0, "gauss"),
    ("T", 7, 0.0, "gauss"),
    ("cross", 31, -100.0, "gauss"),
]


def _problem(shape, n, kappa, kind, seed=0):
    if kind == "manufactured":
        return workloads.manufactured_problem(shape, n, kappa)
    if kind == "shifted":
        return workloads.manufactured_problem(shape, n, kappa, shifted=True)
    return workloads.gaussian_problem(shape, n, kappa, 1, seed, 0)


@pytest.fixture(params=["fft", "auto"])
def dst_algo(request, monkeypatch):
    """Workgroup-wide row FFT with the FFT line kernel, and the automatic
    choice (wave-parallel row FFT, dense line operators)."""
    monkeypatch.setenv("FDS_DST_ALGO", request.param)
    if request.param == "fft":
        monkeypatch.setenv("FDS_LINES", "fft")
    return request.param


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("shape,n,kappa,kind", CASES_SMALL)
def test_small_parity(shape, n, kappa, kind, precision, dst_algo):
    fds = _fds()
    log(f"solve {shape} n={n} kappa={kappa} {kind} prec={precision}")
    prob = _problem(shape, n, kappa, kind)
    ref = oracle_solution(prob)
    plan, rhs, bc, x = device_problem(prob, restart_m=30, precision=precision)
    res = fds.solve(plan, rhs, x, 1e-12, bc=bc)
    assert res.status == 0, res
    err = compare(prob, x, ref)
    log(f"  its={res.iterations} cycles={res.cycles} err={err:.3e} relres={res.relres_schur:.2e} "
        f"global={res.relres_global:.2e}")
    assert err <= 1e-10
    assert res.relres_schur <= 1e-12
    assert res.relres_global <= 1e-11


@pytest.mark.parametrize("kappa,kind", [(0.0, "manufactured"), (-50.0, "gauss")])
def test_full_size_plain_fp64(kappa, kind):
    """The plain method at its full size: cross, 256x256 per square."""
    fds = _fds()
    log(f"full-size n=256 kappa={kappa} {kind}")
    prob = _problem("cross", 256, kappa, kind, seed=3)
    ref = oracle_solution(prob, method="band")
    plan, rhs, bc, x = device_problem(prob, restart_m=30)
    res = fds.solve(plan, rhs, x, 1e-12, bc=bc)
    err = compare(prob, x, ref)
    log(f"  its={res.iterations} err={err:.3e} relres={res.relres_schur:.2e}")
    assert res.status == 0
    assert err <= 1e-10


@pytest.mark.parametrize("restart_m", [6, 16, 30, 40])
@pytest.mark.parametrize("shape,n,kappa,kind", [("cross", 64, 0.0, "shifted"), ("T", 45, -50.0, "gauss"),
                                                ("L", 1, 0.0, "shifted")])
def test_lagged_gram_columns(shape, n, kappa, kind, restart_m, monkeypatch):
    """Plain method with the Gram columns taken from the update pass
    (restart length <= 32) and with the two-pass Gram-Schmidt: both reach the
    oracle, with the same iteration counts up to rounding effects."""
    fds = _fds()
    prob = _problem(shape, n, kappa, kind)
    ref = oracle_solution(prob)
    out = {}
    for lag in ("1", "0"):
        monkeypatch.setenv("FDS_GRAM_LAG", lag)
        log(f"lagged Gram {lag}: {shape} n={n} kappa={kappa} {kind} m={restart_m}")
        plan, rhs, bc, x = device_problem(prob, restart_m=restart_m)
        res = fds.solve(plan, rhs, x, 1e-12, bc=bc)
        err = compare(prob, x, ref)
        log(f"  its={res.iterations} cycles={res.cycles} err={err:.3e} relres={res.relres_schur:.2e}")
        assert res.status == 0, res
        assert err <= 1e-10
        out[lag] = res.iterations
    assert abs(out["1"] - out["0"]) <= max(2, out["0"] // 20), out


@pytest.mark.parametrize("seg", ["8,4", "8,8", "8,16", "16,4", "16,16", "32,4", "32,8", "64,4", "16,32"])
@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("shape,n,kappa,kind", [("cross", 64, 0.0, "shifted"), ("T", 45, -50.0, "gauss")])
def test_tridiag_segment_configs(shape, n, kappa, kind, precision, seg, monkeypatch):
    """Every instantiated (modes per block, rows per segment) pair of the
    segmented tridiagonal solve, forced through its tuning override: full and
    ragged last segments (45 rows), both precisions (32-row segments exist
    for FP32 only; FP64 then keeps the automatic choice)."""
    fds = _fds()
    monkeypatch.setenv("FDS_TRI_SEG", seg)
    log(f"tridiag segments {seg}: {shape} n={n} kappa={kappa} {kind} prec={precision}")
    prob = _problem(shape, n, kappa, kind)
    ref = oracle_solution(prob)
    plan, rhs, bc, x = device_problem(prob, restart_m=30, precision=precision)
    res = fds.solve(plan, rhs, x, 1e-12, bc=bc)
    err = compare(prob, x, ref)
    log(f"  its={res.iterations} cycles={res.cycles} err={err:.3e} relres={res.relres_schur:.2e}")
    assert res.status == 0, res
    assert err <= 1e-10


@pytest.mark.parametrize("shape,n", [("cross", 16), ("L", 20)])
def test_no_preconditioner_baseline(shape, n):
    """P = I (flexible GMRES with z = v) reaches the oracle too, and the
    A_c^-1 preconditioner cuts the iteration count several times over
    (Section 3.2 reports more than sevenfold)."""
    fds = _fds()
    prob = _problem(shape, n, 0.0, "shifted")
    ref = oracle_solution(prob)
    its = {}
    for prec in (fds.NO_PRECOND, fds.FP64):
        log(f"{shape} n={n} precision={prec}")
        plan, rhs, bc, x = device_problem(prob, restart_m=30, precision=prec, max_cycles=400)
        res = fds.solve(plan, rhs, x, 1e-12, bc=bc)
        err = compare(prob, x, ref)
        log(f"  its={res.iterations} cycles={res.cycles} err={err:.3e} stop={res.stop_reason}")
        assert res.status == 0, res
        assert err <= 1e-10
        its[prec] = res.iterations
    assert its[fds.NO_PRECOND] >= 3 * its[fds.FP64], its


@pytest.mark.parametrize("shape,n,kappa", [("cross", 16, 0.0), ("T", 20, -40.0), ("L", 33, 0.0)])
def test_jacobi_preconditioner(shape, n, kappa):
    """P = diag(L_c) (Section 3.2's Jacobi baseline) reaches the oracle's
    solution; its iteration count matches the oracle's own Jacobi-preconditioned
    GMRES (same restart length and stopping rule) to within the FP32 storage
    of z, and stays several times above the A_c^-1 preconditioner's."""
    from oracle import schur
    fds = _fds()
    prob = _problem(shape, n, kappa, "shifted")
    ref = oracle_solution(prob)
    its = {}
    for prec in (fds.JACOBI, fds.FP64):
        log(f"{shape} n={n} kappa={kappa} precision={prec}")
        plan, rhs, bc, x = device_problem(prob, restart_m=30, precision=prec, max_cycles=400)
        res = fds.solve(plan, rhs, x, 1e-12, bc=bc)
        err = compare(prob, x, ref)
        log(f"  its={res.iterations} cycles={res.cycles} err={err:.3e} stop={res.stop_reason}")
        assert res.status == 0, res
        assert err <= 1e-10
        its[prec] = res.iterations
    P = schur.partition(prob.rects, prob.h, kappa, prob.f_grid, prob.g_grid)
    op = schur.SchurOperator(P)
    o = schur.gmres_right(op.apply_L, op.apply_Jinv, op.fprime(), m=30, tol=1e-12, max_cycles=400)
    log(f"  oracle Jacobi GMRES its={o.iterations}")
    assert o.converged
    assert abs(its[fds.JACOBI] - o.iterations) <= max(3, 0.1 * o.iterations), (its, o.iterations)
    assert its[fds.JACOBI] >= 3 * its[fds.FP64], its


def test_solution_is_second_order():
    """Manufactured solution through the whole GPU path: error falls 4x per
    halving of h."""
    fds = _fds()
    errs = []
    for N in (16, 32, 64):
        prob = workloads.manufactured_problem("cross", N - 1, 0.0, shifted=True)
        plan, rhs, bc, x = device_problem(prob)
        res = fds.solve(plan, rhs, x, 1e-12, bc=bc)
        assert res.status == 0
        from oracle import layout as olayout, composite
        g = composite.classify(prob.rects)
        G = olayout.from_user(prob.rects, x.cpu().numpy(), (g.height, g.width))
        m = g.unknown
        errs.append(np.max(np.abs(G[m] - prob.p_exact[:g.height, :g.width][m])))
    for a, b in zip(errs, errs[1:]):
        assert 3.6 < a / b < 4.4, errs


def test_geometry_errors():
    fds = _fds()
    N = 9
    bad = [
        [(0, 0, N, N), (N - 2, 0, 2 * N, N)],                       # overlap
        [(N, N, 2 * N, 2 * N), (2 * N, N, 3 * N, 2 * N - 1)],        # partial side
        # four coupled rectangles (a 2x2 block) that do not form a straight chain
        [(N, N, 2 * N, 2 * N), (N, 2 * N, 2 * N, 3 * N), (2 * N, N, 3 * N, 2 * N),
         (2 * N, 2 * N, 3 * N, 3 * N)],
        [(N, N, 2 * N, 2 * N), (2 * N, N, 3 * N, 2 * N), (2 * N, N - 1, 3 * N, N)],  # arm on arm
        [(0, 0, 1, 5)],                                            # no interior node
    ]
    for rects in bad:
        with pytest.raises(fds.FdsError) as ei:
            fds.Plan(rects, 1.0 / N, 0.0)
        assert ei.value.status == -2, rects


def test_kappa_positive_paths():
    fds = _fds()
    n = 8
    rects = workloads.shape_rects("cross", n)
    h = 1.0 / (n + 1)
    # small positive kappa keeps every mode diagonally dominant: accepted
    fds.Plan(rects, h, 1.0)
    # kappa equal to minus the smallest eigenvalue of a square: singular
    lam = (2 * np.cos(np.pi * h) - 2) / h ** 2 * 2
    with pytest.raises(fds.FdsError) as ei:
        fds.Plan(rects, h, -lam)
    assert ei.value.status == -4
    # a larger kappa makes the lowest sine mode oscillatory
    with pytest.raises(fds.FdsError) as ei:
        fds.Plan(rects, h, -0.8 * lam)
    assert ei.value.status == -3


def test_nonfinite_and_not_converged():
    fds = _fds()
    prob = workloads.gaussian_problem("cross", 16, 0.0, 2, 0, 0)
    plan, rhs, bc, x = device_problem(prob)
    rhs[5] = float("nan")
    res = fds.solve(plan, rhs, x, 1e-12, bc=bc)
    assert res.status == -7
    plan, rhs, bc, x = device_problem(prob, restart_m=2, max_cycles=1)
    res = fds.solve(plan, rhs, x, 1e-12, bc=bc)
    assert res.status == -6
    assert res.cycles == 1 and res.iterations <= 2
    assert np.all(np.isfinite(x.cpu().numpy()))


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_matches_standalone(precision):
    """Each problem of a mixed batch (shapes, sizes, kappa) gives the same
    result as when solved alone."""
    fds = _fds()
    specs = [("cross", 24, 0.0, "gauss", 0), ("L", 40, -70.0, "gauss", 1), ("T", 9, -5.0, "shifted", 0),
             ("cross", 64, -20.0, "gauss", 2), ("square", 30, 0.0, "gauss", 3)]
    probs = [_problem(s, n, k, kind, seed) for (s, n, k, kind, seed) in specs]
    alone = []
    for p in probs:
        plan, rhs, bc, x = device_problem(p, precision=precision)
        r = fds.solve(plan, rhs, x, 1e-11, bc=bc)
        assert r.status == 0
        alone.append((x.clone(), r))
    items = [device_problem(p, precision=precision) for p in probs]
    res = fds.solve_batch([it[0] for it in items], [it[1] for it in items], [it[3] for it in items],
                          [1e-11] * len(items), bcs=[it[2] for it in items])
    for (x_alone, r_alone), it, r in zip(alone, items, res):
        assert r.status == 0
        assert r.iterations == r_alone.iterations
        assert torch.equal(it[3], x_alone)
    # the FP64 bar for both variants: the FP32 preconditioner only changes
    # the basis, the residual and the update are FP64 (relative residual
    # 1e-11 gives solution errors well below 1e-10 at these sizes)
    for p, it in zip(probs, items):
        err = compare(p, it[3], oracle_solution(p))
        log(f"batch {p.shape} n={p.n} precision={precision}: err={err:.3e}")
        assert err <= 1e-10


def test_restart_many_cycles_batch_matches_alone():
    """Short restarts (many cycles) on large centres, second in a batch: the
    restart decision is taken once per problem before V[0] is scaled, so the
    result equals the solve alone bitwise.  (Every block deciding for itself
    while one block updated the cycle count and the previous residual let
    late blocks skip the scaling from the third cycle on.)"""
    fds = _fds()
    first = _problem("L", 640, -30.0, "gauss", 7)
    second = _problem("T", 600, 0.0, "gauss", 8)
    a = device_problem(second, restart_m=6)
    ra = fds.solve(a[0], a[1], a[3], 1e-10, bc=a[2])
    assert ra.cycles >= 4
    items = [device_problem(first, restart_m=6), device_problem(second, restart_m=6)]
    rs = fds.solve_batch([i[0] for i in items], [i[1] for i in items], [i[3] for i in items],
                         [1e-10, 1e-10], bcs=[i[2] for i in items])
    log(f"restart batch: alone {ra.iterations} its / {ra.cycles} cycles, batch {rs[1].iterations}")
    assert rs[1].iterations == ra.iterations
    assert torch.equal(items[1][3], a[3])


@pytest.mark.parametrize("flags,precision", [(0, 0), (0, 1), (1, 0)])
def test_cycle_graphs_match_kernel_launches(monkeypatch, flags, precision):
    """One hipGraph per GMRES cycle (FDS_GRAPH=1, captured after the first
    cycle of a batch and replayed for every later one, with the engine's own
    synchronisations between replays) gives bitwise the result of the cycles
    launched kernel by kernel, and the oracle's solution.  Plain, flexible
    and interface Krylov paths, restart length 6 so the graph is replayed
    many times."""
    fds = _fds()
    probs = [_problem("cross", 40, -10.0, "gauss", 4), _problem("T", 33, 0.0, "shifted", 0)]
    out = {}
    for g in ("0", "1"):
        monkeypatch.setenv("FDS_GRAPH", g)
        items = [device_problem(p, restart_m=6, precision=precision) for p in probs]
        if flags:
            items = []
            for p in probs:
                plan0, rhs, bc, x = device_problem(p, restart_m=6, precision=precision)
                items.append((fds.Plan(p.rects, p.h, p.kappa, restart_m=6, precision=precision,
                                       flags=flags), rhs, bc, x))
        res = fds.solve_batch([i[0] for i in items], [i[1] for i in items], [i[3] for i in items],
                              [1e-11] * len(items), bcs=[i[2] for i in items])
        assert all(r.status == 0 for r in res), res
        assert min(r.cycles for r in res) >= 4
        out[g] = ([i[3].clone() for i in items], [r.iterations for r in res])
        log(f"graphs={g} flags={flags} precision={precision}: its {out[g][1]}")
    assert out["0"][1] == out["1"][1]
    for a, b in zip(out["0"][0], out["1"][0]):
        assert torch.equal(a, b)
    for p, x in zip(probs, out["1"][0]):
        assert compare(p, x, oracle_solution(p)) <= 1e-10


def _drain(srv, tickets, timeout=90.0):
    import time
    results = {}
    t0 = time.time()
    while len(results) < len(tickets) and time.time() - t0 < timeout:
        for t in tickets:
            if t not in results:
                r = srv.poll(t)
                if r is not None:
                    results[t] = r
        time.sleep(0.002)
    return results


def _server_check(prob, x_server, precision, **opts):
    """A server result: bitwise the solve alone (same options), and the
    oracle's solution at the FP64 bar."""
    fds = _fds()
    plan, rhs, bc, x = device_problem(prob, precision=precision, **opts)
    fds.solve(plan, rhs, x, 1e-11, bc=bc)
    assert torch.equal(x, x_server)
    err = compare(prob, x_server, oracle_solution(prob))
    log(f"  {prob.label} {prob.shape} n={prob.n}: err vs oracle {err:.3e}")
    assert err <= 1e-10


def test_server_continuous_batching_matches_alone():
    """Requests that arrive while another is iterating join the running batch
    at a cycle boundary (mixed shapes, sizes and both precisions).  A long
    first request (short restarts, many cycles) is seen running before the
    others are submitted; the server counts their admissions as mid-flight,
    they finish before it, and every result is bitwise the result of the same
    solve alone and matches the oracle."""
    import time
    fds = _fds()
    long_req = _problem("cross", 256, 0.0, "gauss", 1)
    later = [_problem("L", 33, -10.0, "gauss", 5), _problem("cross", 20, 0.0, "shifted", 0),
             _problem("T", 24, -50.0, "gauss", 3), _problem("T", 40, -20.0, "gauss", 2)]
    items, precs, opts, tickets = [], [], [], []
    for k, p in enumerate(later):
        prec = k % 2
        # the FP64 ones share the long request's options and size class, so
        # they join its engine at a cycle boundary; the others start a group
        # of their own beside it
        o = dict(restart_m=6, max_cycles=400) if prec == 0 else {}
        items.append(device_problem(p, precision=prec, **o))
        precs.append(prec)
        opts.append(o)
    first = device_problem(long_req, restart_m=6, precision=0, max_cycles=400)
    # warm the per-length tables and kernels of the later requests
    for it in items:
        fds.solve(it[0], it[1], it[3], 1e-11, bc=it[2])
        it[3].fill_(float("nan"))
    srv = fds.Server(hbm_budget_bytes=1 << 32, max_slots=8)
    t_long = srv.submit(first[0], first[1], first[3], 1e-11, bc=first[2])
    t0 = time.time()
    while True:
        st = srv.stats()
        if st["running"] >= 1 and st["cycles"] >= 2:
            break
        assert time.time() - t0 < 60, st
        time.sleep(0.0002)
    for plan, rhs, bc, x in items:
        tickets.append(srv.submit(plan, rhs, x, 1e-11, bc=bc))
    order = []
    results = {}
    t0 = time.time()
    while len(results) < len(tickets) + 1 and time.time() - t0 < 90:
        for t in tickets + [t_long]:
            if t not in results:
                r = srv.poll(t)
                if r is not None:
                    results[t] = r
                    order.append(t)
        time.sleep(0.001)
    stats = srv.stats()
    srv.close()
    log(f"server stats {stats}; finish order {order}")
    assert len(results) == len(tickets) + 1
    assert stats["admitted_mid_flight"] >= len(later), stats
    assert order[-1] == t_long, order
    assert results[t_long].cycles >= 4, results[t_long]
    assert stats["completed"] == len(later) + 1
    for k, (p, it, t) in enumerate(zip(later, items, tickets)):
        assert results[t].status == 0
        assert results[t].seconds > 0
        _server_check(p, it[3], precs[k], **opts[k])
    assert results[t_long].status == 0
    plan, rhs, bc, x = device_problem(long_req, restart_m=6, precision=0, max_cycles=400)
    fds.solve(plan, rhs, x, 1e-11, bc=bc)
    assert torch.equal(x, first[3])
    assert compare(long_req, first[3], oracle_solution(long_req, method="band")) <= 1e-10


def test_server_reads_inputs_after_the_submitting_stream():
    """Inputs written asynchronously on the caller's stream just before submit
    (no host synchronisation) are read only after that work completed."""
    fds = _fds()
    prob = _problem("cross", 48, -5.0, "gauss", 6)
    plan, rhs, bc, x = device_problem(prob)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    srv = fds.Server(hbm_budget_bytes=1 << 30, max_slots=2)
    with torch.cuda.stream(s):
        big = torch.empty(1 << 26, dtype=torch.float64, device="cuda")
        staged = torch.zeros_like(rhs)
        for _ in range(4):
            big.normal_()            # keep the stream busy before the copy
        staged.copy_(rhs)
        t = srv.submit(plan, staged, x, 1e-11, bc=bc)
    r = _drain(srv, [t])
    srv.close()
    assert r[t].status == 0
    _server_check(prob, x, 0)


def test_server_completion_queue():
    """fds_batch_wait_any hands out every finished request exactly once, each
    matching the oracle, and times out with nothing left."""
    fds = _fds()
    probs = [_problem("cross", 20, 0.0, "gauss", s) for s in range(2)] + \
            [_problem("L", 33, -10.0, "gauss", 5), _problem("T", 120, 0.0, "shifted", 0)]
    srv = fds.Server(hbm_budget_bytes=1 << 31, max_slots=4)
    items = [device_problem(p) for p in probs]
    tickets = [srv.submit(it[0], it[1], it[3], 1e-11, bc=it[2]) for it in items]
    got = {}
    while len(got) < len(tickets):
        r = srv.wait_any(60.0)
        assert r is not None
        t, res = r
        assert t in tickets and t not in got
        got[t] = res
    assert srv.wait_any(0.01) is None
    srv.close()
    for p, it, t in zip(probs, items, tickets):
        assert got[t].status == 0
        _server_check(p, it[3], 0)


def test_server_admission_by_footprint():
    """A budget that holds one problem runs the stream one at a time."""
    fds = _fds()
    probs = [_problem("cross", 24, 0.0, "gauss", s) for s in range(3)]
    items = [device_problem(p) for p in probs]
    one = items[0][0].footprint
    srv = fds.Server(hbm_budget_bytes=int(one * 1.5), max_slots=8)
    tickets = [srv.submit(it[0], it[1], it[3], 1e-11, bc=it[2]) for it in items]
    results = _drain(srv, tickets)
    stats = srv.stats()
    srv.close()
    assert len(results) == len(tickets)
    assert stats["peak_bytes_in_use"] <= int(one * 1.5), stats
    for p, it, t in zip(probs, items, tickets):
        assert results[t].status == 0
        _server_check(p, it[3], 0)


def test_server_results_match_direct():
    fds = _fds()
    probs = [_problem("cross", 20, 0.0, "gauss", s) for s in range(3)] + \
            [_problem("L", 33, -10.0, "gauss", 5), _problem("T", 12, 0.0, "shifted", 0)]
    srv = fds.Server(hbm_budget_bytes=1 << 30, max_slots=3)
    items = [device_problem(p) for p in probs]
    tickets = [srv.submit(it[0], it[1], it[3], 1e-11, bc=it[2]) for it in items]
    results = _drain(srv, tickets, timeout=60)
    srv.close()
    assert len(results) == len(tickets)
    for p, it, t in zip(probs, items, tickets):
        assert results[t].status == 0
        _server_check(p, it[3], 0)
