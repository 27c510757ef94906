"""Parity of single hot-path kernels (through the C ABI) with the oracle."""

import numpy as np
import pytest

import workloads
from oracle import rect, schur
from tests.gpu_util import log

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _fds():
    import paper_2509_23180_amd as fds
    return fds


def _maxprime(N):
    p, best, n = 2, 1, N
    while n > 1 and p * p <= n:
        while n % p == 0:
            best, n = max(best, p), n // p
        p += 1
    return max(best, n)


def _tol64(n):
    # rounding of a mixed-radix FFT grows like log2(N); a generic prime pass of
    # length p adds about p roundings per output
    return 1e-13 * (1 + _maxprime(n + 1) / 32) * max(1.0, np.log2(n + 1) / 8)


# covers mixed radix (e.g. 33 = 3*11), Rader (prime n+1: 17, 97, 101, 257, 1201) and
# Bluestein (n+1 = 301, 1501, 2049) schedules
DST_SIZES = [1, 2, 3, 4, 5, 7, 10, 16, 31, 32, 33, 63, 64, 65, 96, 100, 127, 128, 129, 255, 256, 257,
             300, 511, 512, 1000, 1023, 1024, 1025, 1200, 1500, 2047, 2048]


@pytest.fixture(params=["wave", "wavebig", "fft", "gemm"])
def dst_algo(request, monkeypatch):
    """Every row-transform algorithm: wave-parallel LDS FFT with a row per
    wavefront ("wave", where its radices and register budget allow) or a row
    per workgroup with the tables in global memory ("wavebig"), else the
    workgroup FFT; the workgroup-wide LDS FFT; and the matrix-core product
    (n <= 512)."""
    monkeypatch.setenv("FDS_DST_ALGO", request.param)
    return request.param


@pytest.mark.parametrize("n", DST_SIZES)
def test_dst_rows_fp64(n, dst_algo):
    fds = _fds()
    rows = 17 if n < 1024 else 5
    log(f"dst fp64 n={n} rows={rows}")
    x = np.random.default_rng(n).normal(size=(rows, n))
    ref = rect.dst1_rows(x)
    xi = torch.tensor(x, device="cuda")
    out = torch.empty_like(xi)
    fds.dst_rows(xi, out)
    err = np.abs(out.cpu().numpy() - ref).max() / np.abs(ref).max()
    assert err <= _tol64(n), err
    # in place and scaled
    fds.dst_rows(xi, xi, scale=2.0 / (n + 1))
    back = rect.dst1_rows(xi.cpu().numpy())
    assert np.abs(back - x).max() <= 10 * _tol64(n) * np.abs(x).max()


@pytest.mark.parametrize("n", [1, 7, 16, 32, 33, 64, 100, 255, 256, 257, 300, 1023, 1024, 1200, 2047,
                               2048])
def test_dst_rows_fp32(n, dst_algo):
    fds = _fds()
    log(f"dst fp32 n={n}")
    x = np.random.default_rng(n + 5).normal(size=(9, n)).astype(np.float32)
    ref = rect.dst1_rows(x.astype(np.float64))
    xi = torch.tensor(x, device="cuda")
    out = torch.empty_like(xi)
    fds.dst_rows(xi, out)
    err = np.abs(out.cpu().numpy() - ref).max() / np.abs(ref).max()
    assert err <= 5e-6 * (1 + _maxprime(n + 1) / 32), err


# 1024 rows: the segmented solve's 64 segments of 16 rows x 16 modes (1024
# threads); 2048 rows: FP32 segments of 32 rows, FP64 the unsegmented solve
@pytest.mark.parametrize("rows,modes", [(1, 1), (2, 3), (5, 64), (33, 32), (257, 256), (1025, 300),
                                        (64, 1024), (1024, 1024), (1024, 33), (2048, 128), (2049, 64)])
@pytest.mark.parametrize("kappa", [0.0, -50.0])
def test_tridiag_modes(rows, modes, kappa):
    fds = _fds()
    log(f"tridiag rows={rows} modes={modes} kappa={kappa}")
    h = 1.0 / (modes + 1)
    F = np.random.default_rng(rows * 7 + modes).normal(size=(rows, modes))
    diag = rect.mode_diagonal(modes, h, kappa)
    ref = rect.tridiag_solve_modes(0.5 * F, diag, 1.0 / h ** 2)
    d = torch.tensor(F, device="cuda")
    fds.tridiag_modes(d, h, kappa, scale=0.5)
    err = np.abs(d.cpu().numpy() - ref).max() / np.abs(ref).max()
    # backward-stable solve: relative error up to about u times
    # the condition number of the worst mode's matrix (closed-form spectrum:
    # a_k + 2 delta cos(j pi/(rows+1))), about 2e5 at 1024 rows and kappa 0
    delta = 1.0 / h ** 2
    c = 2 * delta * np.cos(np.pi / (rows + 1)) if rows > 1 else 0.0
    cond = float(np.max((np.abs(diag) + c) / (np.abs(diag) - c)))
    assert err <= max(1e-11, 2 * np.finfo(float).eps * cond), (err, cond)
    d32 = torch.tensor(F, dtype=torch.float32, device="cuda")
    fds.tridiag_modes(d32, h, kappa, scale=0.5)
    err32 = np.abs(d32.double().cpu().numpy() - ref).max() / np.abs(ref).max()
    assert err32 <= 2e-4, err32


@pytest.mark.parametrize("rows,cols", [(1, 1), (2, 3), (5, 7), (32, 32), (33, 32), (256, 256),
                                       (257, 256), (100, 1024)])
@pytest.mark.parametrize("kappa", [0.0, -37.5])
def test_rect_solve(rows, cols, kappa, dst_algo):
    fds = _fds()
    log(f"rect_solve {rows}x{cols} kappa={kappa}")
    h = 1.0 / (max(rows, cols) + 1)
    F = np.random.default_rng(rows + 3 * cols).normal(size=(rows, cols))
    ref = rect.rect_solve(F, h, kappa)
    f = torch.tensor(F, device="cuda")
    z = torch.empty_like(f)
    fds.rect_solve(f, z, h, kappa, precision=fds.FP64)
    err = np.abs(z.cpu().numpy() - ref).max() / np.abs(ref).max()
    assert err <= 1e-11, err
    fds.rect_solve(f, z, h, kappa, precision=fds.FP32_PRECOND)
    err32 = np.abs(z.cpu().numpy() - ref).max() / np.abs(ref).max()
    assert err32 <= 5e-4, err32


@pytest.mark.parametrize("shape", ["cross", "L", "T", "pair", "square"])
@pytest.mark.parametrize("n", [1, 5, 32])
@pytest.mark.parametrize("kappa", [0.0, -50.0])
def test_centre_operator(shape, n, kappa):
    fds = _fds()
    log(f"operator {shape} n={n} kappa={kappa}")
    prob = workloads.gaussian_problem(shape, n, kappa, 11, 0, 0)
    P = schur.partition(prob.rects, prob.h, kappa, prob.f_grid, prob.g_grid)
    op = schur.SchurOperator(P)
    z = np.random.default_rng(n).normal(size=P.centre.size)
    ref = op.apply_L(z)
    plan = fds.Plan(prob.rects, prob.h, kappa)
    zd = torch.tensor(z, device="cuda")
    w = torch.empty_like(zd)
    fds.centre_operator(plan, zd, w)
    err = np.abs(w.cpu().numpy() - ref).max() / np.abs(ref).max()
    assert err <= 1e-12, err


@pytest.mark.parametrize("k,length", [(1, 1), (1, 100), (5, 4097), (30, 65536 + 17), (40, 3000)])
def test_arnoldi_mgs(k, length):
    fds = _fds()
    log(f"arnoldi k={k} len={length}")
    rng = np.random.default_rng(k + length)
    if length >= k:
        Q = np.linalg.qr(rng.normal(size=(length, k)))[0].T
    else:
        pytest.skip("k > len")
    w = rng.normal(size=length)
    h_ref, v_ref = schur.mgs_step(Q, w)
    V = torch.tensor(np.vstack([Q, w[None, :]]), device="cuda").contiguous()
    h = torch.zeros(k + 1, dtype=torch.float64, device="cuda")
    fds.arnoldi_mgs(V, k, h)
    assert np.abs(h.cpu().numpy() - h_ref).max() <= 1e-12 * np.abs(h_ref).max()
    assert np.abs(V[k].cpu().numpy() - v_ref).max() <= 1e-12
