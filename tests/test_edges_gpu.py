"""Empty and degenerate single-problem calls on the GPU: n = 0 and m = n = 0
factorizations are no-ops, tsqr_factor with n > 64 is caqr_factor with
nb = 64, a panel as wide as the matrix is the TSQR itself, apply_q with k = 0
and ls_solve with nrhs = 0 do nothing, square and 1 x 1 problems."""
import numpy as np
import pytest
import torch

import oracle
from paper_1303_5837_amd import caqr, inputs
from tests._gpu import banner, caqr_gpu, factored, require_gpu, tsqr_gpu

pytestmark = pytest.mark.gpu


def test_empty_factorizations():
    require_gpu()
    banner("edge: empty factorizations")
    A = inputs.gaussian(100, 3, 501)
    dA = caqr.fortran(A)
    for fn in (lambda t: caqr.tsqr(t[:, :0]), lambda t: caqr.caqr(t[:, :0], nb=64)):
        F = fn(dA)
        torch.cuda.synchronize()
        assert F.info().panels == 0
    assert np.array_equal(dA.cpu().numpy(), A)  # untouched
    Z = torch.zeros((1, 1), dtype=torch.float64, device="cuda")[:0, :0]
    for fn in (caqr.tsqr, lambda t: caqr.caqr(t, nb=64)):
        F = fn(Z)
        torch.cuda.synchronize()
        assert F.info().m == 0 and F.info().n == 0


def test_tsqr_wider_than_one_panel_is_caqr():
    require_gpu()
    banner("edge: tsqr n > 64")
    A = inputs.gaussian(3000, 100, 502)
    F1, R1 = tsqr_gpu(A)
    F2, R2 = caqr_gpu(A, nb=64)
    assert F1.info().panels == 2 and F1.info().nb == 64
    assert np.array_equal(factored(F1), factored(F2))
    assert oracle.rel_fro(R1, oracle.qr_r(A)) <= 1e-11


def test_single_full_width_panel_is_the_tsqr():
    require_gpu()
    A = inputs.gaussian(5000, 48, 503)
    F1, R1 = tsqr_gpu(A)
    F2, R2 = caqr_gpu(A, nb=48)
    assert F2.info().panels == 1
    assert np.array_equal(factored(F1), factored(F2))


def test_apply_q_and_ls_with_nothing_to_do():
    require_gpu()
    A = inputs.gaussian(400, 20, 504)
    F, _ = tsqr_gpu(A)
    C = torch.zeros((1, 400), dtype=torch.float64, device="cuda").t()[:, :0]
    for op in (caqr.OP_T, caqr.OP_N):
        F.apply_q(C, op)  # k = 0: nothing enqueued, no error
    dA = caqr.fortran(A)
    B = torch.zeros((1, 400), dtype=torch.float64, device="cuda").t()[:, :0]
    X, info = caqr.ls_solve(dA, B)
    torch.cuda.synchronize()
    assert info.status == 0 and X.shape == (20, 0)


def test_square_and_one_by_one():
    require_gpu()
    banner("edge: square and 1x1")
    rng = np.random.default_rng(505)
    n = 50
    A = rng.standard_normal((n, n)) + n * np.eye(n)
    b = rng.standard_normal((n, 1))
    X, info = caqr.ls_solve(caqr.fortran(A), caqr.fortran(b))
    torch.cuda.synchronize()
    assert info.status == 0
    x_ref, st = oracle.ls(A, b)
    assert st == 0
    assert np.linalg.norm(X.cpu().numpy() - x_ref) <= 1e-12 * np.linalg.norm(x_ref)
    assert oracle.ls_eta(A, X.cpu().numpy(), b) <= 1e-15
    for v in (-3.0, 0.0, 2.5):
        F, R = caqr_gpu(np.array([[v]]), nb=64)
        assert R[0, 0] == abs(v) and F.signs()[0] == (-1.0 if v < 0 else 1.0)
