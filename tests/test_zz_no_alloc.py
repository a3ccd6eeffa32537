"""ls_solve_noalloc (no device allocation; workspace in the library's static
per-GPU scratch array) against ls_solve on the same problems: two calls in a
row, the second smaller, so that the second reuses the scratch array the first
left behind; the oracle's least squares beside both; a problem too large for
the array is rejected before anything is enqueued."""
import numpy as np
import pytest
import torch

import oracle
from paper_1303_5837_amd import caqr, inputs
from tests._gpu import banner, require_gpu

pytestmark = pytest.mark.gpu


def _solve(fn, A, B):
    dA, dB = caqr.fortran(A), caqr.fortran(B)
    X, info = fn(dA, dB)
    torch.cuda.synchronize()
    return X.cpu().numpy(), info.status


def test_noalloc_matches_ls_solve_twice_second_smaller():
    require_gpu()
    oracle.set_threads(16)
    # CAQR path (n > 64, four panels, tickets for the narrow updates), then TSQR path
    for (m, n, k) in [(20000, 200, 2), (3000, 40, 1)]:
        banner(f"ls_solve_noalloc m={m} n={n} nrhs={k}")
        A = inputs.gaussian(m, n, 9100 + n)
        B = inputs.gaussian(m, k, 9200 + n)
        Xp, sp = _solve(caqr.ls_solve, A, B)
        Xn, sn = _solve(caqr.ls_solve_noalloc, A, B)
        assert sp == 0 and sn == 0
        assert oracle.rel_fro(Xn, Xp) <= 1e-12
        Xr, st = oracle.ls(A, B)
        assert st == 0
        assert oracle.rel_fro(Xn, Xr) <= 1e-11
        assert oracle.ls_eta(A, Xn, B) <= 1e-15


def test_noalloc_singular_status_and_size_limit():
    require_gpu()
    A = inputs.gaussian(500, 20, 9300)
    A[:, 7] = 0.0
    dA = caqr.fortran(A)
    _, info = caqr.ls_solve_noalloc(dA, caqr.fortran(np.ones((500, 1))))
    torch.cuda.synchronize()
    assert info.status == 5 and info.index == 7
    big = torch.zeros((64, 1 << 20), dtype=torch.float64, device="cuda").t()  # 1M x 64: workspace above 64 MiB
    b = torch.ones((1, 1 << 20), dtype=torch.float64, device="cuda").t()
    with pytest.raises(caqr.CaqrError) as e:
        caqr.ls_solve_noalloc(big, b)
    assert e.value.code == 4
    torch.cuda.synchronize()
    assert float(b.sum()) == float(1 << 20)  # untouched
