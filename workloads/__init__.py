"""Seeded synthetic workloads for the composite-domain Helmholtz-Poisson solver.

This module only *describes problems*: which rectangles make up a domain, and
the values of the source term f and of the Dirichlet data g at grid nodes.  It
contains none of the solver's arithmetic (no discretisation, no transform, no
Krylov step), so both the CPU oracle and the GPU path can take their inputs
from here without sharing any of the method's code.

Geometry frame.  Unit squares on the frame [0, 3]^2.  A square side carries
n interior nodes, so the node spacing is h = 1/(n+1) and node (i, j) sits at
(i*h, j*h).  Rectangles are given as closed boxes of node indices
(i0, j0, i1, j1); their interior nodes are i0 < i < i1, j0 < j < j1.

  centre C = [1,2]^2, arms W = [0,1]x[1,2], E = [2,3]x[1,2],
  S = [1,2]x[0,1], N = [1,2]x[2,3].
  cross = C+W+E+S+N, L = C+N+E, T = C+W+E+S.

Random draws use numpy's PCG64 seeded by
SeedSequence([20250923, config_id, problem_id, rhs_id]); within one seed the
draw order is: Gaussian centres (rejection sampling), widths, amplitudes.
"""

from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Callable, Dict, List, Sequence, Tuple

import numpy as np

SEED_ROOT = 20250923

SHAPES = ("cross", "L", "T")

# arm name -> unit-square offset (column, row) in the 3x3 frame
_SQUARE = {"C": (1, 1), "W": (0, 1), "E": (2, 1), "S": (1, 0), "N": (1, 2)}
_SHAPE_SQUARES = {
    "cross": ("C", "W", "E", "S", "N"),
    "L": ("C", "N", "E"),
    "T": ("C", "W", "E", "S"),
    "square": ("C",),
    "pair": ("C", "E"),
}

Rect = Tuple[int, int, int, int]


def shape_rects(shape: str, n: int) -> List[Rect]:
    """Closed node boxes (i0, j0, i1, j1) of the squares of `shape`, n interior
    nodes per side.  The centre square is always listed first."""
    if shape not in _SHAPE_SQUARES:
        raise ValueError(f"unknown shape {shape!r}")
    if n < 1:
        raise ValueError("n must be >= 1")
    N = n + 1
    out = []
    for sq in _SHAPE_SQUARES[shape]:
        cx, cy = _SQUARE[sq]
        out.append((cx * N, cy * N, (cx + 1) * N, (cy + 1) * N))
    return out


def shape_squares(shape: str) -> Tuple[str, ...]:
    return _SHAPE_SQUARES[shape]


def frame_nodes(n: int) -> Tuple[np.ndarray, np.ndarray, float]:
    """Coordinates of all nodes of the [0,3]^2 frame: X[j, i], Y[j, i], h."""
    N = n + 1
    h = 1.0 / N
    c = np.arange(3 * N + 1, dtype=np.float64) * h
    X, Y = np.meshgrid(c, c, indexing="xy")
    return X, Y, h


def inside_union(shape: str, x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """True where (x, y) lies in the closed union of the shape's unit squares."""
    m = np.zeros(np.broadcast(x, y).shape, dtype=bool)
    for sq in _SHAPE_SQUARES[shape]:
        cx, cy = _SQUARE[sq]
        m |= (x >= cx) & (x <= cx + 1) & (y >= cy) & (y <= cy + 1)
    return m


# ---------------------------------------------------------------------------
# Manufactured solution  p = sin(pi x) sin(pi y) e^{x+y}
# ---------------------------------------------------------------------------

def manufactured_p(x, y, shift=(0.0, 0.0), xp=np):
    xs = x + shift[0]
    ys = y + shift[1]
    return xp.sin(math.pi * xs) * xp.sin(math.pi * ys) * xp.exp(xs + ys)


def manufactured_f(x, y, kappa, shift=(0.0, 0.0), xp=np):
    """Laplacian of manufactured_p plus kappa*p (continuous, analytic)."""
    xs = x + shift[0]
    ys = y + shift[1]
    e = xp.exp(xs + ys)
    lap = e * (2.0 * (1.0 - math.pi ** 2) * xp.sin(math.pi * xs) * xp.sin(math.pi * ys)
               + 2.0 * math.pi * xp.sin(math.pi * (xs + ys)))
    return lap + kappa * manufactured_p(x, y, shift, xp)


# shift that makes every interface and outer edge carry nonzero values
COUPLING_SHIFT = (0.25, 0.4)


# ---------------------------------------------------------------------------
# Seeded sum-of-Gaussians source
# ---------------------------------------------------------------------------

@dataclass(frozen=True)
class GaussianSource:
    centres: np.ndarray  # (16, 2)
    widths: np.ndarray   # (16,)
    amps: np.ndarray     # (16,)

    def __call__(self, x, y, xp=np):
        f = xp.zeros_like(x)
        for g in range(len(self.amps)):
            cx, cy = float(self.centres[g, 0]), float(self.centres[g, 1])
            w = float(self.widths[g])
            a = float(self.amps[g])
            f = f + a * xp.exp(-((x - cx) ** 2 + (y - cy) ** 2) / (2.0 * w * w))
        return f


def rng_for(config_id: int, problem_id: int, rhs_id: int = 0) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([SEED_ROOT, config_id, problem_id, rhs_id]))


def gaussian_source(shape: str, config_id: int, problem_id: int, rhs_id: int,
                    count: int = 16) -> GaussianSource:
    """16 Gaussians, centres uniform over the composite area (rejection from
    the [0,3]^2 frame), widths U[0.05, 0.2], amplitudes N(0, 1)."""
    rng = rng_for(config_id, problem_id, rhs_id)
    centres = np.empty((count, 2))
    k = 0
    while k < count:
        c = rng.uniform(0.0, 3.0, size=2)
        if inside_union(shape, c[0], c[1]):
            centres[k] = c
            k += 1
    widths = rng.uniform(0.05, 0.2, size=count)
    amps = rng.normal(0.0, 1.0, size=count)
    return GaussianSource(centres, widths, amps)


# ---------------------------------------------------------------------------
# Whole problems on the frame grid
# ---------------------------------------------------------------------------

@dataclass
class Problem:
    shape: str
    n: int
    kappa: float
    rects: List[Rect]
    h: float
    f_grid: np.ndarray        # (3N+1, 3N+1) source term at every frame node
    g_grid: np.ndarray        # (3N+1, 3N+1) Dirichlet data at every frame node
    p_exact: np.ndarray = None  # analytic solution on the frame, if known
    label: str = ""


def manufactured_problem(shape: str, n: int, kappa: float = 0.0, shifted: bool = False) -> Problem:
    X, Y, h = frame_nodes(n)
    shift = COUPLING_SHIFT if shifted else (0.0, 0.0)
    p = manufactured_p(X, Y, shift)
    f = manufactured_f(X, Y, kappa, shift)
    return Problem(shape, n, float(kappa), shape_rects(shape, n), h, f, p.copy(), p,
                   label=f"manufactured{'-shifted' if shifted else ''}")


def gaussian_problem(shape: str, n: int, kappa: float, config_id: int, problem_id: int,
                     rhs_id: int) -> Problem:
    X, Y, h = frame_nodes(n)
    src = gaussian_source(shape, config_id, problem_id, rhs_id)
    f = src(X, Y)
    g = np.zeros_like(f)
    return Problem(shape, n, float(kappa), shape_rects(shape, n), h, f, g, None,
                   label=f"gauss[{config_id},{problem_id},{rhs_id}]")


# ---------------------------------------------------------------------------
# Chains of rectangles (several coupled subdomains)
# ---------------------------------------------------------------------------

def chain_rects(n: int, lengths: Sequence[int], vertical: bool = True) -> List[Rect]:
    """A straight chain of rectangles, n interior nodes across; rectangle k
    spans lengths[k] node intervals along the chain.  Listed in chain order
    from the origin; every rectangle except the two ends shares edges with
    two others, so those are the coupled subdomains."""
    N = n + 1
    out, at = [], 0
    for L in lengths:
        if L < 2:
            raise ValueError("every rectangle needs an interior node")
        out.append((0, at, N, at + L) if vertical else (at, 0, at + L, N))
        at += L
    return out


def rects_problem(rects: Sequence[Rect], h: float, kappa: float, kind: str = "shifted",
                  seed: int = 0) -> Problem:
    """Problem on an arbitrary concatenation: the manufactured solution
    (kind "manufactured" / "shifted") or a seeded sum of 16 Gaussians with
    zero Dirichlet data (kind "gauss"; config id 5, centres by rejection from
    the bounding box into the union of the closed rectangles)."""
    I = max(r[2] for r in rects)
    J = max(r[3] for r in rects)
    X, Y = np.meshgrid(np.arange(I + 1) * h, np.arange(J + 1) * h, indexing="xy")
    label = f"{kind}"
    if kind in ("manufactured", "shifted"):
        shift = COUPLING_SHIFT if kind == "shifted" else (0.0, 0.0)
        pe = manufactured_p(X, Y, shift)
        return Problem("rects", 0, float(kappa), list(rects), h, manufactured_f(X, Y, kappa, shift),
                       pe.copy(), pe, label=label)
    if kind != "gauss":
        raise ValueError(f"unknown kind {kind!r}")
    rng = rng_for(5, seed, 0)
    boxes = [(r[0] * h, r[1] * h, r[2] * h, r[3] * h) for r in rects]
    centres = np.empty((16, 2))
    k = 0
    while k < 16:
        c = rng.uniform((0.0, 0.0), (I * h, J * h))
        if any(b[0] <= c[0] <= b[2] and b[1] <= c[1] <= b[3] for b in boxes):
            centres[k] = c
            k += 1
    src = GaussianSource(centres, rng.uniform(0.05, 0.2, size=16), rng.normal(0.0, 1.0, size=16))
    f = src(X, Y)
    return Problem("rects", 0, float(kappa), list(rects), h, f, np.zeros_like(f), None,
                   label=f"gauss[5,{seed},0]")


# ---------------------------------------------------------------------------
# Batched and served workloads
# ---------------------------------------------------------------------------

@dataclass(frozen=True)
class ProblemSpec:
    shape: str
    n: int
    kappa: float
    config_id: int
    problem_id: int
    rhs_id: int

    def build(self) -> Problem:
        return gaussian_problem(self.shape, self.n, self.kappa, self.config_id,
                                self.problem_id, self.rhs_id)


def batch_workload(n_problems: int = 64, rhs_per_problem: int = 8,
                   sizes: Sequence[int] = (64, 128, 256, 512),
                   config_id: int = 3) -> List[ProblemSpec]:
    """64 composite problems: shape uniform over {cross, L, T}, n uniform over
    `sizes`, kappa uniform in [-100, 0]; 8 Gaussian right-hand sides each."""
    out = []
    for p in range(n_problems):
        rng = rng_for(config_id, p, 1 << 20)
        kappa = float(rng.uniform(-100.0, 0.0))
        shape = SHAPES[int(rng.integers(0, 3))]
        n = int(sizes[int(rng.integers(0, len(sizes)))])
        for r in range(rhs_per_problem):
            out.append(ProblemSpec(shape, n, kappa, config_id, p, r))
    return out


@dataclass(frozen=True)
class Request:
    arrival_s: float
    spec: ProblemSpec


def request_stream(rate_per_s: float, duration_s: float, n_min: int = 64, n_max: int = 2048,
                   config_id: int = 4, seed: int = 0) -> List[Request]:
    """Poisson arrivals; shape uniform over {cross, L, T}; n log-uniform in
    [n_min, n_max]; kappa = 0 with probability 1/2 else U[-100, 0]."""
    rng = rng_for(config_id, seed, 1 << 21)
    t = 0.0
    out = []
    k = 0
    ratio = n_max / n_min
    while True:
        t += float(rng.exponential(1.0 / rate_per_s))
        if t > duration_s:
            break
        shape = SHAPES[int(rng.integers(0, 3))]
        n = int(round(n_min * ratio ** float(rng.uniform())))
        kappa = 0.0 if rng.uniform() < 0.5 else float(rng.uniform(-100.0, 0.0))
        out.append(Request(t, ProblemSpec(shape, n, kappa, config_id, k, 0)))
        k += 1
    return out
