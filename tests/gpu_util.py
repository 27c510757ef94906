"""Shared helpers of the GPU parity tests (test infrastructure)."""

import sys

import numpy as np

import workloads
from oracle import composite, layout as olayout


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def device_problem(prob, restart_m=30, precision=0, max_cycles=200, with_bc=True):
    """Plan + device rhs/bc/x for a workloads.Problem (packing through the
    oracle's own layout so a layout bug in the library shows up)."""
    import torch
    import paper_2509_23180_amd as fds
    plan = fds.Plan(prob.rects, prob.h, prob.kappa, restart_m=restart_m, max_cycles=max_cycles,
                    precision=precision)
    rhs = torch.tensor(olayout.to_user(prob.rects, prob.f_grid), dtype=torch.float64, device="cuda")
    bc = None
    if with_bc:
        bc = torch.tensor(olayout.bc_boxes(prob.rects, prob.g_grid), dtype=torch.float64, device="cuda")
    x = torch.full((plan.n_unknowns,), float("nan"), dtype=torch.float64, device="cuda")
    assert rhs.numel() == plan.n_unknowns
    if bc is not None:
        assert bc.numel() == plan.n_bc
    return plan, rhs, bc, x


def oracle_solution(prob, method="auto"):
    return composite.solve(prob.rects, prob.h, prob.kappa, prob.f_grid, prob.g_grid, method=method)


def compare(prob, x_dev, sol):
    """max|x - p*| / max|p*| over all unknowns (global grid comparison)."""
    x = x_dev.detach().cpu().numpy()
    H, W = sol.grid.height, sol.grid.width
    G = olayout.from_user(prob.rects, x, (H, W))
    ref = sol.on_grid()
    m = sol.grid.unknown
    assert np.all(np.isfinite(G[m]))
    return float(np.max(np.abs(G[m] - ref[m])) / max(np.max(np.abs(ref[m])), 1e-300))
