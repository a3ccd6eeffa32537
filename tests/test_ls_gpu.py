"""Least squares through the factorization, vs the oracle and the exact construction."""
import numpy as np
import pytest
import torch

import oracle
from paper_1303_5837_amd import caqr, inputs
from tests._gpu import require_gpu

pytestmark = pytest.mark.gpu


def _solve(A, B):
    dA, dB = caqr.fortran(A), caqr.fortran(B)
    X, info = caqr.ls_solve(dA, dB)
    torch.cuda.synchronize()
    return X.cpu().numpy(), info


@pytest.mark.parametrize("m,n,nrhs", [(2000, 30, 1), (5000, 64, 3), (3000, 200, 2), (1500, 1024, 1)])
def test_ls_matches_oracle(m, n, nrhs):
    require_gpu()
    A = inputs.gaussian(m, n, 3000 + n)
    B = inputs.gaussian(m, nrhs, 4000 + n)
    X, info = _solve(A, B)
    assert info.status == 0
    Xref, st = oracle.ls(A, B)
    assert st == 0
    assert oracle.rel_fro(X, Xref) <= 1e-11
    assert oracle.ls_eta(A, X, B) <= 1e-15


def test_consistent_system_and_conditioning():
    require_gpu()
    rng = np.random.default_rng(7)
    m, n = 4000, 100
    U = np.linalg.qr(rng.standard_normal((m, n)))[0]
    V = np.linalg.qr(rng.standard_normal((n, n)))[0]
    for kappa in (1e2, 1e6):
        s = inputs.geometric_singular_values(n, kappa)
        A = (U * s) @ V.T
        xt = rng.standard_normal(n)
        X, info = _solve(A, A @ xt)
        assert info.status == 0
        assert np.linalg.norm(X[:, 0] - xt) / np.linalg.norm(xt) <= 50 * kappa * 2.0 ** -53 * n
        assert oracle.ls_eta(A, X, A @ xt, norm_a=1.0) <= 1e-15


def test_singular_and_nonfinite():
    require_gpu()
    A = inputs.gaussian(500, 20, 8)
    A[:, 5] = 0.0
    _, info = _solve(A, np.ones((500, 1)))
    assert info.status == 5 and info.index == 5
    A = inputs.gaussian(500, 20, 9)
    A[3, 3] = np.inf
    _, info = _solve(A, np.ones((500, 1)))
    assert info.status == 6
