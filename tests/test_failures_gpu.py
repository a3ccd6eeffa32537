"""Host-forced failures through the C ABI (no GPU fault involved): a workspace
limit below what a call needs gives CAQR_ERR_ALLOC with nothing enqueued, and a
forced device error at a chosen launch site surfaces as CAQR_ERR_DEVICE from
the call that reached it, after which the handle still computes the oracle's
result."""
import numpy as np
import pytest
import torch

import oracle
from paper_1303_5837_amd import caqr, inputs
from tests._gpu import banner, caqr_gpu, require_gpu

pytestmark = pytest.mark.gpu


def test_workspace_limit_gives_alloc_error():
    require_gpu()
    banner("failures: workspace limit")
    h = caqr.handle(0)
    A = inputs.gaussian(2000, 100, 601)
    b = inputs.gaussian(2000, 1, 602)
    try:
        h.set_workspace_limit(4096)
        for call in (lambda t: caqr.caqr(t, nb=64), lambda t: caqr.tsqr(t[:, :40]),
                     lambda t: caqr.ls_solve(t, caqr.fortran(b)), lambda t: caqr.tsqr_batched([t[:, :16]])):
            dA = caqr.fortran(A)
            before = dA.clone()
            with pytest.raises(caqr.CaqrError) as e:
                call(dA)
            assert e.value.code == 2
            torch.cuda.synchronize()
            assert torch.equal(dA, before)  # nothing was enqueued
    finally:
        h.set_workspace_limit(0)
    F, R = caqr_gpu(A)
    assert oracle.rel_fro(R, oracle.qr_r(A)) <= 1e-11


def test_forced_device_error_propagates():
    require_gpu()
    banner("failures: forced device errors")
    h = caqr.handle(0)
    A = inputs.gaussian(3000, 300, 603)
    # caqr_factor of 3000 x 300, nb 64: panel + T of panel 0, then for each of
    # the next four panels the narrow update, the wide update (none before the
    # last panel, whose columns are all that is left), the panel and its T:
    # 17 launch sites
    try:
        for k in (1, 2, 3, 4, 7, 12, 17):
            dA = caqr.fortran(A)
            h.fail_at(k)
            with pytest.raises(caqr.CaqrError) as e:
                caqr.caqr(dA, nb=64)
            assert e.value.code == 3, k
            torch.cuda.synchronize()
        h.fail_at(18)  # one past the last site: the factorization completes
        F, R = caqr_gpu(A)
        h.fail_at(0)
        assert oracle.rel_fro(R, oracle.qr_r(A)) <= 1e-11
        C = caqr.fortran(inputs.gaussian(3000, 2, 604))
        h.fail_at(1)
        with pytest.raises(caqr.CaqrError) as e:
            F.apply_q(C, caqr.OP_T)
        assert e.value.code == 3
        h.fail_at(1)
        with pytest.raises(caqr.CaqrError) as e:
            caqr.tsqr_batched([caqr.fortran(A[:, :32])])
        assert e.value.code == 3
        h.fail_at(3)  # ls_solve of n <= 64: the panel, Q^T b (T first), then the back substitution
        with pytest.raises(caqr.CaqrError) as e:
            caqr.ls_solve(caqr.fortran(A[:, :50]), caqr.fortran(A[:, 50:51]))
        assert e.value.code == 3
    finally:
        h.fail_at(0)
    torch.cuda.synchronize()
    F, R = caqr_gpu(A)  # the handle is still usable
    assert oracle.rel_fro(R, oracle.qr_r(A)) <= 1e-11
    x, info = caqr.ls_solve(caqr.fortran(A[:, :50]), caqr.fortran(A[:, 50:51]))
    torch.cuda.synchronize()
    xr, st = oracle.ls(A[:, :50], A[:, 50:51])
    assert info.status == 0 and st == 0
    assert oracle.rel_fro(x.cpu().numpy(), xr) <= 1e-11
