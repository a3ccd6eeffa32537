"""Mixed-precision least squares (trailing-update products with the leaf
reflectors on FP32 MFMA, FP64 refinement): every solution against the oracle's
least squares within the perturbation bound of its conditioning and within the
backward-error target eta <= 1e-12 (the pinned measure), on the mixed-precision
configuration's construction A = U diag(s) V^T with kappa up to 1e6; the
unrefined FP32-update solution at FP32 accuracy (a wrong FP32 product would
show here); the FP64 fallback bitwise equal to the plain solve; statuses."""
import numpy as np
import pytest
import torch

import oracle
from paper_1303_5837_amd import caqr, inputs
from tests._gpu import banner, require_gpu

pytestmark = pytest.mark.gpu

U64 = 2.0 ** -53


def forward_bound(A, R, x, b, eps_mult=10):
    """Twice the first-order perturbation bound of two backward-stable
    solutions (relative backward error 10 n u), floored at 1e-11; kappa from
    the singular values of the oracle's R (those of A)."""
    sv = np.linalg.svd(R, compute_uv=False)
    kappa = sv[0] / sv[-1]
    eps = eps_mult * A.shape[1] * U64
    r = b - A @ x
    bound = eps * kappa * (2 + (kappa + 1) * np.linalg.norm(r, axis=0).max() / (sv[0] * np.linalg.norm(x)))
    return max(1e-11, 2 * bound), kappa


def solve(A, B, **kw):
    dA, dB = caqr.fortran(A), caqr.fortran(B)
    dA0 = dA.clone()
    X, info = caqr.ls_solve(dA, dB, **kw)
    torch.cuda.synchronize()
    if kw.get("precision", 0) == caqr.LS_MIXED_F32:
        assert torch.equal(dA, dA0)  # A is only read
    return X.cpu().numpy(), info


@pytest.mark.parametrize("m,n,nrhs,kappa", [(20000, 300, 1, 1e2), (20000, 300, 2, 1e4), (20000, 300, 1, 1e6),
                                            (65536, 1024, 1, 1e2), (65536, 1024, 1, 1e6), (3000, 129, 3, 1e5)])
def test_mixed_against_oracle(m, n, nrhs, kappa):
    require_gpu()
    oracle.set_threads(16)
    banner(f"mixed ls m={m} n={n} nrhs={nrhs} kappa={kappa:.0e}")
    A = inputs.conditioned_host(m, n, kappa, 5000 + n + int(np.log10(kappa)))
    B = inputs.gaussian(m, nrhs, 5100 + n)
    X, info = solve(A, B, precision=caqr.LS_MIXED_F32)
    banner(f"  status {info.status} iters {info.iters} fallback {info.fallback} eta bound {info.eta:.2e}")
    assert info.status == 0 and info.fallback == 0
    assert info.eta <= 1e-12
    f = oracle.qr(A)
    Xr, st = oracle.ls(A, B)
    assert st == 0
    tol, kap = forward_bound(A, f.R, Xr, B)
    err = oracle.rel_fro(X, Xr)
    eta = oracle.ls_eta(A, X, B, norm_a=1.0)
    banner(f"  vs oracle {err:.2e} (bound {tol:.1e}, kappa {kap:.1e}); eta {eta:.2e}")
    assert err <= tol
    assert eta <= 1e-12
    assert eta <= info.eta * (1 + 1e-6)  # the reported bound is an upper bound


def test_unrefined_fp32_update_at_fp32_accuracy():
    """One refinement step only (no fallback): the solution of the FP32-update
    factorization is already accurate to about kappa u32; a wrong FP32 product
    or lane layout would leave it at O(1)."""
    require_gpu()
    A = inputs.conditioned_host(8000, 256, 1e2, 5200)
    B = inputs.gaussian(8000, 1, 5201)
    X, info = solve(A, B, precision=caqr.LS_MIXED_F32, max_iter=1, tol=1e-300, fallback=False)
    assert info.status == 7  # CAQR_ERR_NOT_CONVERGED with the last iterate
    Xr, _ = oracle.ls(A, B)
    err = oracle.rel_fro(X, Xr)
    banner(f"  one step: vs oracle {err:.2e}")
    assert err <= 1e2 * 2.0 ** -24 * 100


def test_fallback_is_the_fp64_solve():
    """An unreachable tolerance: refinement stalls, the FP64 solve of A replaces
    it (flagged), bitwise the plain ls_solve; small n is the FP64 solve."""
    require_gpu()
    A = inputs.conditioned_host(5000, 200, 1e3, 5300)
    B = inputs.gaussian(5000, 2, 5301)
    X, info = solve(A, B, precision=caqr.LS_MIXED_F32, tol=1e-300, max_iter=6)
    assert info.status == 0 and info.fallback == 1
    Xp, ip = solve(A, B)
    assert ip.status == 0
    assert np.array_equal(X, Xp)
    A2 = inputs.gaussian(3000, 40, 5302)
    X2, i2 = solve(A2, B[:3000], precision=caqr.LS_MIXED_F32)
    Xp2, _ = solve(A2, B[:3000])
    assert i2.status == 0 and np.array_equal(X2, Xp2)


def test_mixed_singular():
    require_gpu()
    A = inputs.gaussian(3000, 100, 5400)
    A[:, 70] = 0.0
    _, info = solve(A, np.ones((3000, 1)), precision=caqr.LS_MIXED_F32)
    assert info.status == 5 and info.index == 70
