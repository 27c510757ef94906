"""The allocation-free Arnoldi step (fds_k_arnoldi_mgs_noalloc) through the C
ABI: results identical to the allocating entry point's on two calls in a row,
the second with a smaller input (the shared working memory keeps the first
call's contents), both checked against the oracle's MGS step; a call beyond
the working memory fails before launching anything."""

import numpy as np
import pytest

from oracle import schur
from tests.gpu_util import log

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _case(k, length, seed):
    rng = np.random.default_rng(seed)
    Q = np.linalg.qr(rng.normal(size=(length, k)))[0].T
    w = rng.normal(size=length)
    return Q, w


def _run(fn, Q, w, k):
    V = torch.tensor(np.vstack([Q, w[None, :]]), device="cuda").contiguous()
    h = torch.full((k + 1,), float("nan"), dtype=torch.float64, device="cuda")
    fn(V, k, h)
    torch.cuda.synchronize()
    return V, h


def test_noalloc_matches_allocating_entry_point():
    import paper_2509_23180_amd as fds
    # first call: 40 vectors of 300,017 (147 blocks: two-level Gram
    # reduction); second call smaller: 7 vectors of 5,000 (one level)
    for k, length, seed in ((40, 300017, 1), (7, 5000, 2)):
        log(f"noalloc Arnoldi k={k} len={length}")
        Q, w = _case(k, length, seed)
        V_ref, h_ref = _run(fds.arnoldi_mgs, Q, w, k)
        V_na, h_na = _run(fds.arnoldi_mgs_noalloc, Q, w, k)
        assert torch.equal(h_na, h_ref), (h_na - h_ref).abs().max()
        assert torch.equal(V_na, V_ref)
        h_or, v_or = schur.mgs_step(Q, w)
        assert np.abs(h_na.cpu().numpy() - h_or).max() <= 1e-12 * np.abs(h_or).max()
        assert np.abs(V_na[k].cpu().numpy() - v_or).max() <= 1e-12


def test_noalloc_rejects_work_beyond_its_memory():
    import paper_2509_23180_amd as fds
    k, length = 120, 1 << 24          # about 62 MB of partials: more than the 8 MiB array
    V = torch.zeros((2, 8), dtype=torch.float64, device="cuda")   # never touched: rejected first
    h = torch.zeros(4, dtype=torch.float64, device="cuda")
    lib = fds.load_library()
    st = lib.fds_k_arnoldi_mgs_noalloc(V.data_ptr(), k, length, h.data_ptr(), None)
    assert st == -5
    assert b"bytes of working memory" in lib.fds_last_error()
