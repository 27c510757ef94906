#!/usr/bin/env python3
"""Benchmark of the FFT-preconditioned interface GMRES on one MI355X.

Default workload ("serving"): a Poisson stream of 200 requests/s, shape
uniform over cross / L / T of unit squares, n log-uniform in [64, 2048]
interior nodes per side, kappa 0 with probability 1/2 else U[-100, 0], seeded
sums of 16 Gaussians as right-hand sides, relative residual 1e-10, replayed
open-loop against the continuous-batching server.  A step is one second of
arrivals (--warmup seconds of warm-up, --steps measured seconds; the
right-hand sides of the whole trace are generated on the device before the
replay, about 4 GB per second of arrivals, so a 60-second window is run with
--serving-paths limited to the headline path).  The
headline path is the interface Krylov iteration, GMRES(80) in FP64; the
mixed-precision FGMRES(40) path and the plain FP64 GMRES(30) path replay the
same trace beside it.  Latency runs from the scheduled arrival to completion.

Prints ONE JSON line (solves/s, p50/p99 latency, roofline of the dominant
kernel, CPU oracle baseline).  Diagnostics go to stderr.

Other workloads (--workload): "plain" (cross of 256x256 per square, 18 solves
per step, GMRES(30) FP64), "interface" (cross of 1024x1024 per square, 4
solves per step, the interface GMRES(80) path without the server), "precision" (cross 1024x1024 per square,
FGMRES(40) with an FP32 preconditioner, error against the SuperLU oracle),
"batching" (64 composite problems x 8 right-hand sides, sizes 64..512,
FGMRES(40); also with cycle graphs and without the transform tuner), "chain"
(four 512x512 squares stacked, two of them coupled, interface GMRES(80), error
against the SuperLU oracle),
"convergence" (iteration counts with P = I, Jacobi and A_c^-1, the iteration
count against n, a restart sweep).
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ("paper_2509_23180_amd/csrc/kernels.hip", "paper_2509_23180_amd/csrc/dst_wave.hip",
                  "paper_2509_23180_amd/csrc/ik_kernels.hip",
                  "paper_2509_23180_amd/csrc/fft_device.h", "paper_2509_23180_amd/csrc/fft_wave.h",
                  "paper_2509_23180_amd/csrc/fds_internal.h")
# kernel class -> name of the HIP kernel that implements it (rocprofv3 summaries)
CLASS_KERNEL = {"dst": "k_dst_wave", "tridiag": "k_tridiag_seg", "operator": "k_operator",
                "gram_dots": "k_gram_dots", "gram_update": "k_gram_update", "lines": "k_lines_dense",
                "cols": "k_idst_cols"}


IK_CLASS_KERNEL = {"gram_dots": "k_ik_wdots", "gram_update": "k_ik_update", "lines": "k_ik_cross", "operator": "k_ik_compose",
                   "other": "k_ik_start", "cols": "k_idst_cols", "tridiag": "k_tridiag_seg",
                   "dst": "k_dst_wave"}


def class_kernel(cls: str, opts: dict) -> str:
    """Kernel of a timing class for a solver configuration: the plain method
    with restart length <= 32 takes its Gram columns from the update pass
    (boundary dots + k_gram_update_lag) unless FDS_GRAM_LAG=0; the interface
    Krylov iteration has kernels of its own."""
    if opts.get("flags", 0) & 1:
        return IK_CLASS_KERNEL.get(cls, cls)
    lag = (opts.get("precision", 0) == 0 and opts.get("restart_m", 30) <= 32
           and os.environ.get("FDS_GRAM_LAG", "1") != "0")
    if lag and cls == "gram_dots":
        return "k_gram_bdots"
    if lag and cls == "gram_update":
        return "k_gram_update_lag"
    return CLASS_KERNEL.get(cls, cls)


def traffic_summary(args) -> None:
    """Per-dispatch HBM bytes of every kernel from two rocprofv3 --pmc runs of
    the workload (FETCH_SIZE, WRITE_SIZE; KiB per dispatch) scaled by the same
    counters on a 1 GiB device copy; writes profiles/traffic_<kernel>_<workload>.json
    for the named kernel (all of its template instantiations) and prints a
    markdown table.  Runs on the host only."""
    import csv
    fetch_dir, write_dir, cfetch_dir, cwrite_dir = args.traffic_summary

    def per_kernel(d, counter):
        out = {}
        with open(os.path.join(d, "run_counter_collection.csv")) as fh:
            for row in csv.DictReader(fh):
                if row["Counter_Name"] != counter:
                    continue
                k = row["Kernel_Name"]
                c = out.setdefault(k, [0, 0.0])
                c[0] += 1
                c[1] += float(row["Counter_Value"])
        return out

    def copy_kib(d, counter):
        # the 1 GiB copy: the largest dispatch of __amd_rocclr_copyBuffer
        best = 0.0
        with open(os.path.join(d, "run_counter_collection.csv")) as fh:
            for row in csv.DictReader(fh):
                if row["Counter_Name"] == counter and "copyBuffer" in row["Kernel_Name"]:
                    best = max(best, float(row["Counter_Value"]))
        return best

    gib = float(1 << 30)
    cf, cw = copy_kib(cfetch_dir, "FETCH_SIZE"), copy_kib(cwrite_dir, "WRITE_SIZE")
    fscale, wscale = gib / (cf * 1024.0), gib / (cw * 1024.0)
    fe, wr = per_kernel(fetch_dir, "FETCH_SIZE"), per_kernel(write_dir, "WRITE_SIZE")

    def short(k):
        k = k.replace("void ", "").replace("fds::", "")
        return k.split("(")[0]

    rows = []
    for k in sorted(fe, key=lambda k: -fe[k][1]):
        n, f = fe[k]
        wn, w = wr.get(k, [n, 0.0])
        rows.append((short(k), n, f / n * 1024 * fscale / 1e6, w / max(wn, 1) * 1024 * wscale / 1e6))
    print(f"calibration: 1 GiB copy reads FETCH_SIZE {cf:.1f} KiB, writes WRITE_SIZE {cw:.1f} KiB "
          f"per dispatch: scales {fscale:.4f} / {wscale:.4f}")
    print("| kernel | dispatches | HBM read MB / dispatch | HBM write MB / dispatch |")
    print("|---|---:|---:|---:|")
    for name, n, f, w in rows[:12]:
        print(f"| {name} | {n} | {f:.2f} | {w:.2f} |")
    sel = [k for k in fe if short(k).startswith(args.traffic_kernel + "<") or short(k) == args.traffic_kernel]
    if not sel:
        print(f"no dispatches of {args.traffic_kernel}", file=sys.stderr)
        sys.exit(1)
    n = sum(fe[k][0] for k in sel)
    fb = sum(fe[k][1] for k in sel) * 1024 * fscale / n
    wn = sum(wr.get(k, [0, 0.0])[0] for k in sel)
    wb = sum(wr.get(k, [0, 0.0])[1] for k in sel) * 1024 * wscale / max(wn, 1)
    rec = {"kernel": args.traffic_kernel, "workload": args.workload,
           "kernel_source_hash": kernel_source_hash(),
           "hbm_bytes_per_launch": round(fb + wb, 1), "fetch_bytes_per_launch": round(fb, 1),
           "write_bytes_per_launch": round(wb, 1), "launches": n,
           "fetch_scale": round(fscale, 4), "write_scale": round(wscale, 4),
           "calibration": f"1 GiB device copy: FETCH_SIZE {cf:.1f} KiB, WRITE_SIZE {cw:.1f} KiB per dispatch"}
    path = os.path.join(ROOT, "profiles", f"traffic_{args.traffic_kernel}_{args.workload}.json")
    with open(path, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec))


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _r(v, d=3):
    return None if v is None else round(v, d)


def pct(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = min(len(xs) - 1, max(0, int(round(q / 100.0 * (len(xs) - 1)))))
    return xs[k]


def stream_ceiling(device):
    """Practical HBM ceilings of this device, measured with plain device
    kernels over 1 GiB FP64 vectors (outside the timed region): a copy, a
    read-only sum and a triad (two reads, one write), in GB/s."""
    import torch
    n = (1 << 30) // 8
    a = torch.ones(n, dtype=torch.float64, device=device)
    b = torch.empty_like(a)
    c = torch.ones_like(a)

    def rate(f, nbytes, reps=10):
        for _ in range(2):
            f()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            f()
        e1.record()
        torch.cuda.synchronize()
        return round(nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9, 1)

    out = {"copy": rate(lambda: b.copy_(a), 16 * n), "read": rate(lambda: a.sum(), 8 * n),
           "triad": rate(lambda: torch.add(a, c, alpha=2.0, out=b), 24 * n)}
    del a, b, c
    torch.cuda.empty_cache()
    return out


def add_practical(roofline, ceiling):
    """The roofline against the measured triad ceiling as well as the
    published peak."""
    if roofline is None or ceiling is None:
        return
    roofline["practical_peak"] = ceiling
    a = roofline.get("achieved")
    roofline["frac_practical"] = round(a / ceiling["triad"], 4) if a and ceiling.get("triad") else None


# --------------------------------------------------------------------------- workloads

def build_workload(name, device):
    """Returns (description dict, list of (plan_key, Problem)), plan kwargs."""
    import workloads
    items = []
    if name == "plain":
        for kappa in (0.0, -50.0):
            items.append(workloads.manufactured_problem("cross", 256, kappa))
            for seed in range(8):
                items.append(workloads.gaussian_problem("cross", 256, kappa, 1, seed, 0))
        desc = {"workload": "cross, 256x256 interior nodes per square (328,704 unknowns per solve), "
                            "plain FP64 GMRES(30), rel-res 1e-10, kappa in {0,-50} x "
                            "{manufactured, 8 seeded Gaussian} right-hand sides",
                "solves_per_step": len(items), "n": 256, "restart_m": 30, "tol": 1e-10,
                "precision": "fp64"}
        opts = dict(restart_m=30, precision=0)
    elif name == "precision":
        items.append(workloads.manufactured_problem("cross", 1024, 0.0))
        items.append(workloads.gaussian_problem("cross", 1024, 0.0, 2, 0, 0))
        desc = {"workload": "cross, 1024x1024 interior nodes per square (5,246,976 unknowns per solve), "
                            "FGMRES(40) with FP32 DST+tridiagonal preconditioner, FP64 Krylov, "
                            "rel-res 1e-10, manufactured and seeded Gaussian right-hand sides",
                "solves_per_step": len(items), "n": 1024, "restart_m": 40, "tol": 1e-10,
                "precision": "fp32-preconditioned"}
        opts = dict(restart_m=40, precision=1)
    elif name == "interface":
        for kappa in (0.0, -50.0):
            items.append(workloads.manufactured_problem("cross", 1024, kappa))
            items.append(workloads.gaussian_problem("cross", 1024, kappa, 2, 0, 0))
        desc = {"workload": "cross, 1024x1024 interior nodes per square (5,246,976 unknowns per solve), "
                            "interface Krylov GMRES(80) in FP64, rel-res 1e-10, kappa in {0,-50} x "
                            "{manufactured, seeded Gaussian} right-hand sides, one batch of 4 solves per step",
                "solves_per_step": len(items), "n": 1024, "restart_m": 80, "tol": 1e-10,
                "precision": "fp64"}
        opts = dict(restart_m=80, precision=0, flags=1)
    elif name == "chain":
        n = 512
        rects = workloads.chain_rects(n, [n + 1] * 4, vertical=True)
        h = 1.0 / (n + 1)
        for kappa in (0.0, -50.0):
            items.append(workloads.rects_problem(rects, h, kappa, "shifted"))
            for seed in (0, 1):
                items.append(workloads.rects_problem(rects, h, kappa, "gauss", seed))
        desc = {"workload": "chain of four 512x512 squares stacked (two coupled, 1,050,112 unknowns "
                            "per solve; coupled block 512 x 1025), interface Krylov GMRES(80) in FP64, "
                            "rel-res 1e-10, kappa in {0,-50} x {manufactured, 2 seeded Gaussian} "
                            "right-hand sides, one batch of 6 solves per step",
                "solves_per_step": len(items), "n": n, "restart_m": 80, "tol": 1e-10,
                "precision": "fp64"}
        opts = dict(restart_m=80, precision=0, flags=1)
    elif name == "batching":
        specs = workloads.batch_workload()
        items = [s.build() for s in specs]
        desc = {"workload": "64 composite problems (cross/L/T, n in {64,128,256,512}, kappa in "
                            "[-100,0]) x 8 seeded Gaussian right-hand sides = 512 solves, "
                            "FGMRES(40) FP32 preconditioner, rel-res 1e-10",
                "solves_per_step": len(items), "restart_m": 40, "tol": 1e-10,
                "precision": "fp32-preconditioned"}
        opts = dict(restart_m=40, precision=1)
    else:
        raise SystemExit(f"unknown workload {name}")
    return desc, items, opts


def to_device(items, opts, device):
    import torch
    import paper_2509_23180_amd as fds
    from paper_2509_23180_amd import layout as playout
    plans = {}
    out = []
    for prob in items:
        key = (tuple(prob.rects), prob.h, prob.kappa)
        if key not in plans:
            plans[key] = fds.Plan(prob.rects, prob.h, prob.kappa, **opts)
        plan = plans[key]
        rhs = torch.tensor(playout.pack_unknowns(prob.rects, prob.f_grid), device=device)
        bc = torch.tensor(playout.pack_boxes(prob.rects, prob.g_grid), device=device)
        x = torch.zeros(plan.n_unknowns, dtype=torch.float64, device=device)
        out.append((plan, rhs, bc, x))
    return plans, out


# --------------------------------------------------------------------------- convergence

def run_convergence(args, device):
    """The paper's convergence comparison on these kernels (Section 3.2): GMRES
    iterations to rel-res 1e-10 without preconditioner (P = I) and with A_c^-1,
    at two n and two restart lengths; the iteration count of the
    preconditioned method against n (power-law fit); and a restart sweep at
    n = 256.  Manufactured solution on the cross, kappa = 0.  One solve per
    case, timed with the device synchronised around it."""
    import math
    import torch
    import workloads
    import paper_2509_23180_amd as fds

    tol = 1e-10

    def one(n, m, precision, max_cycles=200):
        prob = workloads.manufactured_problem("cross", n, 0.0, shifted=True)
        _, dev = to_device([prob], dict(restart_m=m, precision=precision, max_cycles=max_cycles), device)
        plan, rhs, bc, x = dev[0]
        fds.solve(plan, rhs, x, tol, bc=bc)          # tables, tuning, code load
        x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fds.solve(plan, rhs, x, tol, bc=bc)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        stop = r.stop_reason
        log(f"n={n} m={m} precision={precision}: its={r.iterations} cycles={r.cycles} "
            f"relres={r.relres_schur:.2e} stop={stop} {ms:.1f} ms")
        return {"n": n, "m": m, "iterations": r.iterations, "cycles": r.cycles, "status": r.status,
                "stop": stop, "relres": r.relres_schur, "ms": round(ms, 3)}

    compare = []
    for n in (32, 64):
        for m in (30, 80):
            a = one(n, m, fds.NO_PRECOND, max_cycles=400)
            jac = one(n, m, fds.JACOBI, max_cycles=400)
            b = one(n, m, fds.FP64)
            compare.append({"n": n, "m": m, "none": a, "jacobi": jac, "A_c_inv": b,
                            "ratio": round(a["iterations"] / max(1, b["iterations"]), 2),
                            "ratio_jacobi": round(jac["iterations"] / max(1, b["iterations"]), 2)})
    vs_n = [one(n, 30, fds.FP64) for n in (32, 64, 128, 256, 512, 1024)]
    xs = [math.log(r["n"]) for r in vs_n]
    ys = [math.log(max(1, r["iterations"])) for r in vs_n]
    xm, ym = sum(xs) / len(xs), sum(ys) / len(ys)
    slope = sum((x - xm) * (y - ym) for x, y in zip(xs, ys)) / sum((x - xm) ** 2 for x in xs)
    sweep = [one(256, m, fds.FP64) for m in (20, 40, 60, 80, 100, 120)]
    ratios = [c["ratio"] for c in compare if c["none"]["status"] == 0]
    return {
        "metric": "GMRES iterations to rel-res 1e-10: no preconditioner (and Jacobi) over A_c^-1 "
                  "(cross, kappa=0)",
        "value": min(ratios) if ratios else None, "unit": "x (smallest ratio over converged cases)",
        "n_gpus": 1, "steps": 1, "warmup": 1, "ms_per_step": None, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64+f32", "data": "synthetic",
        "config": {"workload": "convergence: cross, manufactured solution, kappa 0, rel-res 1e-10",
                   "compare_P_I_Jacobi_A_c_inv": compare,
                   "iterations_vs_n": {"restart_m": 30, "cases": vs_n,
                                       "fit": f"iterations ~ n^{slope:.3f}"},
                   "restart_sweep_n256": sweep},
        "roofline": None, "cpu_baseline": None,
    }


# --------------------------------------------------------------------------- serving

def request_rhs(spec, device):
    """Right-hand side of one request on the device: the seeded Gaussian
    source evaluated at the owned unknown nodes, rectangle by rectangle in
    the ABI layout (Dirichlet data zero, passed as NULL).  All nodes of the
    request go through one broadcast sum over the Gaussians, in chunks."""
    import torch
    import workloads
    from paper_2509_23180_amd import layout as playout
    n = spec.n
    h = 1.0 / (n + 1)
    rects = workloads.shape_rects(spec.shape, n)
    src = workloads.gaussian_source(spec.shape, spec.config_id, spec.problem_id, spec.rhs_id)
    xs, ys = [], []
    for r in range(len(rects)):
        ilo, ihi, jlo, jhi = playout.owned_box(rects, r)
        gx = torch.arange(ilo, ihi + 1, dtype=torch.float64, device=device) * h
        gy = torch.arange(jlo, jhi + 1, dtype=torch.float64, device=device) * h
        xs.append(gx.repeat(jhi - jlo + 1))
        ys.append(gy.repeat_interleave(ihi - ilo + 1))
    X, Y = torch.cat(xs), torch.cat(ys)
    cx = torch.tensor(src.centres[:, 0], dtype=torch.float64, device=device)[:, None]
    cy = torch.tensor(src.centres[:, 1], dtype=torch.float64, device=device)[:, None]
    iw = torch.tensor(-0.5 / src.widths ** 2, dtype=torch.float64, device=device)[:, None]
    amp = torch.tensor(src.amps, dtype=torch.float64, device=device)[None, :]
    out = torch.empty_like(X)
    chunk = 1 << 22
    for a in range(0, X.numel(), chunk):
        x, y = X[a:a + chunk], Y[a:a + chunk]
        e = torch.exp(((x[None, :] - cx) ** 2 + (y[None, :] - cy) ** 2) * iw)
        out[a:a + chunk] = (amp @ e)[0]
    return rects, h, out


class TimedSlice:
    """Turns per-kernel timing of one class on for a slice of the measured
    window (events on every launch of the class cost a few microseconds of
    dispatch gap, so only a fifth of the window carries them)."""

    def __init__(self, fds, cls, t_on, t_off):
        import threading
        self.fds, self.cls = fds, cls
        self.th = threading.Thread(target=self._run, args=(t_on, t_off), daemon=True)

    def _run(self, t_on, t_off):
        time.sleep(max(0.0, t_on - time.perf_counter()))
        self.fds.timing_enable([self.cls])
        time.sleep(max(0.0, t_off - time.perf_counter()))
        self.fds.timing_enable([])

    def start(self):
        self.th.start()

    def join(self):
        self.th.join()


SUBMITTERS = 4   # front-end threads building plans and submitting requests


class PlanCache:
    """Plans keyed by (shape, n, kappa), the least recently used dropped
    beyond `capacity` (a dropped plan stays alive while a request uses it)."""

    def __init__(self, capacity=256):
        import collections
        self.capacity = capacity
        self.d = collections.OrderedDict()

    def get(self, key):
        p = self.d.get(key)
        if p is not None:
            self.d.move_to_end(key)
        return p

    def put(self, key, plan):
        self.d[key] = plan
        while len(self.d) > self.capacity:
            self.d.popitem(last=False)


def request_inputs(reqs, device):
    """Right-hand sides of every request of a trace, generated on the device
    before the replay (the requests' data is resident in HBM when they
    arrive)."""
    import torch
    out = []
    for rq in reqs:
        rects, h, rhs = request_rhs(rq.spec, device)
        out.append((rects, h, rhs))
    torch.cuda.synchronize()
    return out


def replay(fds, torch, srv, reqs, inputs, opts, device, t_measure, plan_cache, timed=None):
    """Open-loop replay of a request trace against a server.  A submitter
    thread takes each request at its arrival time, builds its plan (or takes
    it from the plan cache) and its output buffer, and submits it with its
    right-hand side (already on the device); the latency clock starts at the
    scheduled arrival.  The main thread collects results from the server's
    completion queue as they are published.  Returns per-request records."""
    import threading
    recs = [None] * len(reqs)
    xs = [None] * len(reqs)
    t0 = time.perf_counter() + 0.2
    lock = threading.Lock()
    k_of = {}     # ticket -> request index
    early = {}    # results collected before their submitter recorded the ticket

    def record(k, t_done, r):
        recs[k].update(done=t_done, status=r.status, iterations=r.iterations, cycles=r.cycles,
                       relres=r.relres_schur, stop=r.stop_reason, server_ms=r.seconds * 1e3,
                       n=reqs[k].spec.n)
        xs[k] = None

    def submitter(first, step):
        torch.cuda.set_device(device)
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            for k in range(first, len(reqs), step):
                rq = reqs[k]
                delay = t0 + rq.arrival_s - time.perf_counter()
                if delay > 0:
                    time.sleep(delay)
                sp = rq.spec
                key = (sp.shape, sp.n, sp.kappa)
                tp = time.perf_counter()
                plan = plan_cache.get(key)
                hit = plan is not None
                rects, h, rhs = inputs[k]
                if plan is None:
                    plan = fds.Plan(rects, h, sp.kappa, **opts)
                    plan_cache.put(key, plan)
                x = torch.empty(plan.n_unknowns, dtype=torch.float64, device=device)
                with lock:
                    recs[k] = {"arrival": t0 + rq.arrival_s, "plan_hit": hit}
                    xs[k] = x
                t = srv.submit(plan, rhs, x, 1e-10, stream=stream)
                with lock:
                    recs[k]["prep_ms"] = (time.perf_counter() - tp) * 1e3
                    k_of[t] = k
                    got = early.pop(t, None)
                    if got is not None:
                        record(k, *got)

    # a front end of SUBMITTERS threads, request k handled by thread k % SUBMITTERS
    ths = [threading.Thread(target=submitter, args=(i, SUBMITTERS)) for i in range(SUBMITTERS)]
    for th in ths:
        th.start()
    if timed is not None:
        timed.start()
    done = 0
    while done < len(reqs):
        got = srv.wait_any(0.05)
        if got is None:
            continue
        t_done = time.perf_counter()
        t, r = got
        with lock:
            k = k_of.get(t)
            if k is None:
                early[t] = (t_done, r)
            else:
                record(k, t_done, r)
        done += 1
    for th in ths:
        th.join()
    if timed is not None:
        timed.join()
    for rq, rec in zip(reqs, recs):
        rec["latency_ms"] = (rec["done"] - rec["arrival"]) * 1e3
        rec["measured"] = rq.arrival_s >= t_measure
    return recs


def latency_by_n(meas):
    """Latency percentiles per octave of n, with the part spent inside the
    server (submission to publication of the result)."""
    out = {}
    for lo in (64, 128, 256, 512, 1024):
        hi = 2 * lo if lo < 1024 else 2049
        sel = [r for r in meas if lo <= r["n"] < hi]
        if not sel:
            continue
        lat = [r["latency_ms"] for r in sel]
        srv = [r["server_ms"] for r in sel]
        out[f"{lo}-{hi - 1}"] = {"requests": len(sel), "p50": _r(pct(lat, 50)), "p99": _r(pct(lat, 99)),
                                 "server_p50": _r(pct(srv, 50)), "server_p99": _r(pct(srv, 99)),
                                 "iterations_mean": round(sum(r["iterations"] for r in sel) / len(sel), 1)}
    return out


def summarise(recs, reqs, srv_stats):
    meas = [r for r in recs if r["measured"]]
    lat = [r["latency_ms"] for r in meas]
    first = min(r["arrival"] for r in meas)
    last = max(r["done"] for r in meas)
    prep = [r["prep_ms"] for r in meas]
    return {"requests": len(meas), "converged": sum(1 for r in meas if r["status"] == 0),
            "throughput_solves_per_s": round(len(meas) / (last - first), 3),
            "makespan_s": round(last - first, 3),
            "latency_ms_p50": _r(pct(lat, 50)), "latency_ms_p99": _r(pct(lat, 99)),
            "latency_ms_max": _r(max(lat)), "latency_ms_mean": _r(sum(lat) / len(lat)),
            "plan_cache_hit_rate": round(sum(1 for r in meas if r["plan_hit"]) / len(meas), 3),
            "request_prep_ms_p50": _r(pct(prep, 50)), "request_prep_ms_p99": _r(pct(prep, 99)),
            "iterations_mean": round(sum(r["iterations"] for r in meas) / len(meas), 1),
            "max_relres_schur": max(r["relres"] for r in meas),
            "admitted_mid_flight": srv_stats["admitted_mid_flight"],
            "server_host_s": {k[5:-2]: round(srv_stats[k], 3) for k in
                              ("host_admit_s", "host_retire_s", "host_tasks_s", "host_launch_s", "host_wait_s")},
            "peak_hbm_gb": round(srv_stats["peak_bytes_in_use"] / 1e9, 2),
            "latency_by_n": latency_by_n(meas),
            "not_converged": [{"shape": reqs[k].spec.shape, "n": reqs[k].spec.n,
                               "kappa": round(reqs[k].spec.kappa, 3), "problem": reqs[k].spec.problem_id,
                               "status": r["status"], "stop": r["stop"], "cycles": r["cycles"],
                               "iterations": r["iterations"], "relres": r["relres"]}
                              for k, r in enumerate(recs) if r["measured"] and r["status"] != 0][:10]}


SERVING_PATHS = {
    # the interface Krylov iteration (FP64, basis on the centre's interface
    # lines); restart length 80 is the paper's best (Section 3.2)
    "interface_gmres80_fp64": dict(restart_m=80, precision=0, flags=1),
    "interface_gmres40_fp64": dict(restart_m=40, precision=0, flags=1),
    # FP32 sine transforms and tridiagonal solves inside flexible GMRES(40)
    "mixed_fgmres40_fp32_precond": dict(restart_m=40, precision=1),
    # the plain method, full centre vectors in FP64
    "plain_gmres30_fp64": dict(restart_m=30, precision=0),
}
DEFAULT_SERVING_PATHS = ["interface_gmres80_fp64", "mixed_fgmres40_fp32_precond", "plain_gmres30_fp64"]


def run_serving(args, device):
    import torch
    import paper_2509_23180_amd as fds
    import workloads
    warm, meas = float(args.warmup), float(args.steps)
    reqs = workloads.request_stream(args.serving_rate, warm + meas, n_min=64, n_max=args.serving_nmax)
    log(f"serving: {len(reqs)} requests at {args.serving_rate:g}/s over {warm:g} s warm-up + {meas:g} s "
        f"measured, n in [64, {args.serving_nmax}]")
    t_in = time.perf_counter()
    inputs = request_inputs(reqs, device)
    log(f"serving: right-hand sides of {len(reqs)} requests generated on the device in "
        f"{time.perf_counter() - t_in:.1f} s")
    # transform tables depend on the length only (not on shape or kappa): a
    # server builds them once for the lengths it serves, before taking
    # requests (like the transform tuning table)
    t_in = time.perf_counter()
    for n in sorted({r.spec.n for r in reqs}):
        x = torch.zeros((1, n), dtype=torch.float64, device=device)
        fds.dst_rows(x, x)
    log(f"serving: transform tables of {len({r.spec.n for r in reqs})} lengths built in "
        f"{time.perf_counter() - t_in:.1f} s")
    out = {}
    headline = "interface_gmres80_fp64"
    roofline = None
    cls_times = None
    names = args.serving_paths.split(",") if args.serving_paths else DEFAULT_SERVING_PATHS
    paths = {k: SERVING_PATHS[k] for k in names}
    if headline not in paths:
        headline = next(iter(paths))
    for name, opts in paths.items():
        # the comparison paths replay the same trace up to the end of its
        # first `--serving-compare-seconds` measured seconds
        span = warm + meas if name == headline else warm + min(meas, args.serving_compare_seconds)
        sub = [r for r in reqs if r.arrival_s <= span]
        sub_in = inputs[:len(sub)]
        srv = fds.Server(hbm_budget_bytes=int(args.serving_budget_gb * (1 << 30)),
                         max_slots=args.serving_slots)
        plan_cache = PlanCache()
        timed = None
        if name == headline:
            # warm-up pass with every class timed: which kernel dominates
            fds.timing_reset()
            fds.timing_enable(None)
            nwarm = sum(1 for r in reqs if r.arrival_s < warm)
            replay(fds, torch, srv, reqs[:nwarm], inputs[:nwarm], opts, device, warm, PlanCache())
            fds.timing_enable([])
            cls_times = {}
            for c in ("dst", "tridiag", "operator", "gram_dots", "gram_update", "lines", "cols", "other"):
                calls, ms, by = fds.timing_read(c)
                cls_times[c] = {"calls": calls, "ms": round(ms, 3),
                                "GB/s": round(by / (ms * 1e-3) / 1e9, 1) if ms > 0 and by > 0 else None}
            dominant = max((c for c in cls_times if c != "other"), key=lambda c: cls_times[c]["ms"])
            log(f"{name}: per-class times over the warm-up: {cls_times}; dominant {dominant}")
            fds.timing_reset()
            t_base = time.perf_counter() + 0.2
            timed = TimedSlice(fds, dominant, t_base + warm + 0.4 * meas, t_base + warm + 0.6 * meas)
        t_wall = time.perf_counter()
        recs = replay(fds, torch, srv, sub, sub_in, opts, device, warm, plan_cache, timed)
        st = srv.stats()
        srv.close()
        out[name] = summarise(recs, sub, st)
        out[name]["trace_s"] = span
        out[name]["wall_s"] = round(time.perf_counter() - t_wall, 2)
        log(f"{name}: {out[name]}")
        if name == headline:
            calls, ms, by = fds.timing_read(dominant)
            kname = class_kernel(dominant, opts)
            achieved = (by / calls) / ((ms / calls) * 1e-3) / 1e9 if calls and ms > 0 else None
            roofline = {"bound": "hbm", "achieved": _r(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved else None,
                        "traffic": None, "kernel": kname, "class": dominant, "launches": calls,
                        "avg_launch_us": round(ms / calls * 1e3, 3) if calls else None,
                        "algorithmic_bytes_per_launch": round(by / calls, 1) if calls else None,
                        "timed_window": "middle fifth of the measured window"}
            tfile = os.path.join(ROOT, "profiles", f"traffic_{kname}_serving.json")
            if os.path.exists(tfile):
                with open(tfile) as fh:
                    tr = json.load(fh)
                if tr.get("kernel_source_hash") == kernel_source_hash():
                    roofline["traffic"] = tr.get("hbm_bytes_per_launch")
        del plan_cache
        torch.cuda.empty_cache()
    del inputs
    torch.cuda.empty_cache()
    add_practical(roofline, stream_ceiling(device))
    head = out[headline]
    cpu = None
    if not args.no_cpu_baseline:
        cpu = serving_cpu_baseline(reqs, args.cpu_seconds)
    return {
        "metric": "solves/s & p50/p99 latency at rel-res 1e-10; DST/Thomas GB/s vs HBM peak",
        "value": head["throughput_solves_per_s"], "unit": "solves/s", "n_gpus": 1,
        "steps": int(meas), "warmup": int(warm),
        "ms_per_step": round(head["makespan_s"] * 1e3 / meas, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"serving: Poisson request stream {args.serving_rate:g}/s, shape U{{cross,L,T}}, "
                               f"n log-uniform [64,{args.serving_nmax}], kappa 0 w.p. 1/2 else U[-100,0], "
                               f"seeded Gaussian RHS, rel-res 1e-10; continuous-batching server "
                               f"({args.serving_slots} slots, {args.serving_budget_gb:g} GB); a step is one "
                               f"second of arrivals ({warm:g} s warm-up, {meas:g} s measured); right-hand sides "
                               f"resident in HBM before the replay; transform tables per length built "
                               f"before it; plans built at arrival inside the latency by "
                               f"{SUBMITTERS} front-end threads (LRU cache of 256 plans)",
                   "headline_path": headline, "paths": out, "latency_ms": {
                       "p50": head["latency_ms_p50"], "p99": head["latency_ms_p99"]}},
        "kernels_warmup": cls_times, "roofline": roofline, "cpu_baseline": cpu,
        "kernel_source_hash": kernel_source_hash(),
    }


def serving_cpu_baseline(reqs, budget_s):
    """The FP64 oracle on requests of the same trace, taken in arrival order
    among those it finishes in seconds (n <= 256), until the time budget is
    spent."""
    from oracle import composite
    try:
        import threadpoolctl
        cores = max([i.get("num_threads", 1) for i in threadpoolctl.threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count()
    # only the oracle's assembly and solve are timed (not the input generation)
    done, probs, dt = [], [], 0.0
    for rq in reqs:
        if rq.spec.n > 256:
            continue
        prob = rq.spec.build()
        t0 = time.perf_counter()
        composite.solve(prob.rects, prob.h, prob.kappa, prob.f_grid, prob.g_grid)
        dt += time.perf_counter() - t0
        done.append(f"{rq.spec.shape} n={rq.spec.n}")
        probs.append(prob)
        if dt > budget_s:
            break
    out = {"value": round(len(done) / dt, 4), "unit": "solves/s", "cores": int(cores), "kind": "oracle",
           "sample": f"{len(done)} requests of the trace in arrival order with n <= 256 "
                     f"({', '.join(done[:6])}{', ...' if len(done) > 6 else ''}); global composite "
                     f"system, LAPACK banded Cholesky; {dt:.1f} s (larger requests excluded: minutes each)",
           "cpu_model": cpu_model()}
    # the same requests with one BLAS thread, for a third of the budget
    try:
        import threadpoolctl
        with threadpoolctl.threadpool_limits(limits=1):
            k, t1 = 0, time.perf_counter()
            for prob in probs:
                composite.solve(prob.rects, prob.h, prob.kappa, prob.f_grid, prob.g_grid)
                k += 1
                if time.perf_counter() - t1 > budget_s / 3:
                    break
            d1 = time.perf_counter() - t1
        out["one_thread"] = {"value": round(k / d1, 4), "cores": 1,
                             "sample": f"the first {k} of the same requests; {d1:.1f} s"}
    except Exception as ex:   # threadpoolctl missing: report the multi-thread figure only
        out["one_thread"] = {"value": None, "sample": f"not measured ({type(ex).__name__})"}
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


# --------------------------------------------------------------------------- reduced precision vs FP64

def precision_error(items, xs):
    """max|x - p*| / max|p*| of every solution of the precision workload
    against the FP64 oracle (sparse direct solve of the global system, one
    factorisation for both right-hand sides of the domain), computed after
    the timed region."""
    import numpy as np
    from oracle import composite, layout as olayout
    prob0 = items[0]
    log(f"error vs the FP64 oracle: SuperLU on {prob0.shape} n={prob0.n} ...")
    t0 = time.perf_counter()
    groups = {}
    for k, p in enumerate(items):
        groups.setdefault((tuple(p.rects), p.h, p.kappa), []).append(k)
    sols = [None] * len(items)
    for (rects, h, kappa), ks in groups.items():
        for k, sol in zip(ks, composite.solve_many(list(rects), h, kappa,
                                                   [(items[k].f_grid, items[k].g_grid) for k in ks],
                                                   method="splu")):
            sols[k] = sol
    dt = time.perf_counter() - t0
    out = {}
    for prob, sol, x in zip(items, sols, xs):
        H, W = sol.grid.height, sol.grid.width
        G = olayout.from_user(prob.rects, x.detach().cpu().numpy(), (H, W))
        ref = sol.on_grid()
        m = sol.grid.unknown
        out[f"{prob.label} kappa={prob.kappa:g}"] = float(np.max(np.abs(G[m] - ref[m])) / np.max(np.abs(ref[m])))
    log(f"error vs oracle: {out} ({dt:.1f} s)")
    return {"max_rel_err": out, "oracle": "global composite system, SuperLU (scipy splu), FP64",
            "oracle_seconds": round(dt, 1)}


# --------------------------------------------------------------------------- CPU baseline

def cpu_baseline(items, sample):
    """The FP64 oracle (banded direct solve of the global system) timed on the
    host cores on a bounded sample of the same workload."""
    from oracle import composite
    try:
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        cores = max([i.get("num_threads", 1) for i in info] + [1])
    except Exception:
        cores = os.cpu_count()
    picks = items[:1] + items[len(items) // 2:len(items) // 2 + 1] if len(items) > 1 else items
    picks = picks[:sample]
    t0 = time.perf_counter()
    for prob in picks:
        composite.solve(prob.rects, prob.h, prob.kappa, prob.f_grid, prob.g_grid)
    dt = time.perf_counter() - t0
    return {"value": round(len(picks) / dt, 6), "unit": "solves/s", "cores": int(cores),
            "kind": "oracle",
            "sample": f"{len(picks)} of the {len(items)} solves of one step "
                      f"({', '.join(p.label + ' kappa=' + str(p.kappa) for p in picks)}); "
                      f"global composite system, LAPACK banded Cholesky; {dt:.1f} s"}


# --------------------------------------------------------------------------- main

def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (serving: seconds of measured arrivals; default 10)")
    ap.add_argument("--warmup", type=int, default=None,
                    help="warm-up steps (serving: seconds of arrivals before the measured window; default 2)")
    ap.add_argument("--workload", default="serving",
                    choices=["serving", "plain", "precision", "batching", "interface", "chain",
                             "convergence"])
    ap.add_argument("--serving-rate", type=float, default=200.0, help="requests per second")
    ap.add_argument("--serving-compare-seconds", type=float, default=5.0,
                    help="measured seconds of the trace replayed on the comparison paths")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="serving: CPU oracle time budget")
    ap.add_argument("--serving-paths", default="",
                    help="comma-separated subset of the serving paths (default: all three)")
    ap.add_argument("--serving-nmax", type=int, default=2048)
    ap.add_argument("--serving-budget-gb", type=float, default=160.0)
    ap.add_argument("--serving-slots", type=int, default=64)
    ap.add_argument("--cpu-sample", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-oracle-error", action="store_true",
                    help="precision and chain workloads: skip the error against the FP64 oracle")
    ap.add_argument("--latency-solves", type=int, default=10)
    ap.add_argument("--roofline-class", default="auto",
                    help="batch workloads: kernel class of the roofline line (default: the dominant one)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of 1 GiB (HBM counter calibration)")
    ap.add_argument("--traffic-summary", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR",
                                                            "COPY_WRITE_DIR"),
                    help="host only: turn rocprofv3 --pmc output directories into the traffic record")
    ap.add_argument("--traffic-kernel", default="k_gram_update_lag")
    args = ap.parse_args()
    if args.steps is None:
        args.steps = 10
    if args.warmup is None:
        args.warmup = 2
    if args.traffic_summary:
        traffic_summary(args)
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: every solve of this method fits one MI355X, and "
              "runs on several GPUs are not implemented (independent problems would shard across "
              "GPUs with no communication).", file=sys.stderr)
        sys.exit(2)

    # measured transform choices of this device kind (see tune.cpp): plans
    # built as requests arrive then cost no device measurement
    table = os.path.join(ROOT, "paper_2509_23180_amd", "tune_gfx950.txt")
    if "FDS_TUNE_FILE" not in os.environ and os.path.exists(table):
        os.environ["FDS_TUNE_FILE"] = table
    import torch
    import paper_2509_23180_amd as fds
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    device = "cuda:0"
    torch.cuda.set_device(0)

    if args.copy_calibration:
        n = (1 << 30) // 8
        a = torch.ones(n, dtype=torch.float64, device=device)
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = 20
        for _ in range(reps):
            b.copy_(a)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        print(json.dumps({"copy_bytes_per_launch": 2 * n * 8, "GB/s": 2 * n * 8 * reps / dt / 1e9}))
        return

    if args.workload == "convergence":
        print(json.dumps(run_convergence(args, device)), flush=True)
        return

    if args.workload == "serving":
        print(json.dumps(run_serving(args, device)), flush=True)
        return

    desc, items, opts = build_workload(args.workload, device)
    log(f"building {len(items)} problems on {device}")
    plans, dev = to_device(items, opts, device)
    P = [d[0] for d in dev]
    R = [d[1] for d in dev]
    B = [d[2] for d in dev]
    X = [d[3] for d in dev]
    tol = desc["tol"]
    T = [tol] * len(dev)

    def step():
        return fds.solve_batch(P, R, X, T, bcs=B)

    for w in range(args.warmup):
        res = step()
        log(f"warmup {w}: iterations {[r.iterations for r in res][:6]}...")

    # per-class totals of one step with every class timed -> dominant class
    fds.timing_reset()
    fds.timing_enable(None)
    step()
    fds.timing_enable([])
    classes = {}
    for name in ("dst", "tridiag", "operator", "gram_dots", "gram_update", "lines", "cols", "other"):
        c, ms, by = fds.timing_read(name)
        classes[name] = {"calls": c, "ms": round(ms, 4),
                         "GB/s": round(by / (ms * 1e-3) / 1e9, 1) if ms > 0 and by > 0 else None}
    dominant = max((k for k in classes if k != "other"), key=lambda k: classes[k]["ms"])
    log(f"per-class (one step, all classes timed): {classes}; dominant: {dominant}")
    if args.roofline_class != "auto":
        dominant = args.roofline_class

    # timed region: the dominant class carries HIP events (on the stream it is
    # launched on) in one of the timed steps, the middle one.  Every step is
    # the same work; an event pair around a launch adds a few microseconds of
    # dispatch gap, which timing every step would charge to the throughput.
    fds.timing_reset()
    ev_step = args.steps // 2
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    step_ms = []
    results = None
    for k in range(args.steps):
        if k == ev_step:
            fds.timing_enable([dominant])
        t0 = time.perf_counter()
        results = step()
        step_ms.append((time.perf_counter() - t0) * 1e3)
        if k == ev_step:
            fds.timing_enable([])
    torch.cuda.synchronize()
    total = time.perf_counter() - t_start
    fds.timing_enable([])
    calls, ms, algo_bytes = fds.timing_read(dominant)
    solves = len(dev) * args.steps
    value = solves / total
    ok = all(r.status == 0 and r.relres_schur <= tol for r in results)
    its = [r.iterations for r in results]
    log(f"timed: {args.steps} steps in {total:.3f} s -> {value:.2f} solves/s; iterations {its}")

    # single-solve latency (outside the timed region)
    lat = []
    for _ in range(args.latency_solves):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fds.solve(P[0], R[0], X[0], tol, bc=B[0])
        lat.append((time.perf_counter() - t0) * 1e3)

    # batching: the same steps with one hipGraph per cycle and with the static
    # transform choice instead of the autotuner's (both are read when a batch
    # is set up, so they apply from the next step on)
    variants = None
    if args.workload == "batching":
        variants = {"default_graphs_off_tuned": round(value, 3)}
        for label, env in (("graphs_on", {"FDS_GRAPH": "1"}),
                           ("untuned_transforms", {"FDS_DST_TUNE": "0"}),
                           ("graphs_on_untuned", {"FDS_GRAPH": "1", "FDS_DST_TUNE": "0"})):
            saved = {k: os.environ.get(k) for k in env}
            os.environ.update(env)
            step()
            torch.cuda.synchronize()
            k_steps = max(1, min(args.steps, 3))
            t0 = time.perf_counter()
            for _ in range(k_steps):
                step()
            torch.cuda.synchronize()
            variants[label] = round(len(dev) * k_steps / (time.perf_counter() - t0), 3)
            for k, v in saved.items():
                if v is None:
                    os.environ.pop(k, None)
                else:
                    os.environ[k] = v
            log(f"variant {label}: {variants[label]} solves/s")

    error_vs_oracle = None
    if args.workload in ("precision", "chain") and not args.no_oracle_error:
        error_vs_oracle = precision_error(items, X)

    achieved = (algo_bytes / calls) / ((ms / calls) * 1e-3) / 1e9 if calls and ms > 0 else None
    traffic = None
    kname = class_kernel(dominant, opts)
    tfile = os.path.join(ROOT, "profiles", f"traffic_{kname}_{args.workload}.json")
    if os.path.exists(tfile):
        with open(tfile) as fh:
            tr = json.load(fh)
        if tr.get("kernel_source_hash") == kernel_source_hash():
            traffic = tr.get("hbm_bytes_per_launch")
    roofline = {"bound": "hbm", "achieved": round(achieved, 1) if achieved else None,
                "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved else None,
                "traffic": traffic,
                "kernel": kname,
                "launches": calls, "event_steps": 1,
                "avg_launch_us": round(ms / calls * 1e3, 3) if calls else None,
                "algorithmic_bytes_per_launch": round(algo_bytes / calls, 1) if calls else None}

    add_practical(roofline, stream_ceiling(device))
    cpu = None
    if not args.no_cpu_baseline and args.cpu_sample > 0:
        log("timing the CPU oracle on a bounded sample ...")
        cpu = cpu_baseline(items, args.cpu_sample)

    line = {
        "metric": "solves/s & p50/p99 latency at rel-res 1e-10; DST/Thomas GB/s vs HBM peak",
        "value": round(value, 3), "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(total / args.steps * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic", "config": desc,
        "converged": ok, "iterations": its,
        "latency_ms": {"step_p50": _r(pct(step_ms, 50)), "step_p99": _r(pct(step_ms, 99)),
                       "single_solve_p50": _r(pct(lat, 50)), "single_solve_p99": _r(pct(lat, 99))},
        "kernels": classes,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "kernel_source_hash": kernel_source_hash(),
    }
    if error_vs_oracle is not None:
        line["error_vs_oracle"] = error_vs_oracle
    if variants is not None:
        line["variants_solves_per_s"] = variants
    if args.workload not in ("plain", "interface", "chain"):
        line["dtype"] = "f64+f32"
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
