"""Batched least squares (n_i <= 64): each problem against the oracle's least
squares and against the plain ls_solve (the batched solve applies Q^T with the
stored reflectors one at a time, the plain one with compact WY, so the two agree
to rounding), backward error eta, statuses, and problems with nothing to do."""
import numpy as np
import pytest
import torch

import oracle
from paper_1303_5837_amd import caqr, inputs
from tests._gpu import banner, require_gpu

pytestmark = pytest.mark.gpu

# (m, n, nrhs): TSQR trees of several depths, ragged leaves, m == n, n on and
# off 16-column blocks, several right-hand sides, empty problems
MIX = [(2000, 30, 1), (5000, 64, 3), (257, 33, 2), (64, 64, 1), (100, 8, 1), (40000, 17, 1), (1500, 1, 2),
       (3000, 0, 1), (500, 20, 0), (9000, 48, 1), (70000, 64, 1)]


def make(mix, seed):
    As, Bs = [], []
    for i, (m, n, k) in enumerate(mix):
        As.append(inputs.gaussian(m, n, seed + i) if n else np.zeros((m, 0)))
        Bs.append(inputs.gaussian(m, k, seed + 100 + i) if k else np.zeros((m, 0)))
    return As, Bs


def dev(x):
    if x.shape[1] == 0:
        return torch.empty((0, x.shape[0]), dtype=torch.float64, device="cuda").t()
    return caqr.fortran(x)


def run(mix, seed, **plan):
    As, Bs = make(mix, seed)
    dA, dB = [dev(a) for a in As], [dev(b) for b in Bs]
    Xs, info = caqr.ls_solve_batched(dA, dB, **plan)
    torch.cuda.synchronize()
    return As, Bs, [x.cpu().numpy() for x in Xs], info


def test_batched_ls_against_oracle_and_plain():
    require_gpu()
    oracle.set_threads(16)
    As, Bs, Xs, info = run(MIX, 8100)
    for i, (m, n, k) in enumerate(MIX):
        banner(f"batched ls {i}: m={m} n={n} nrhs={k} info={info[i]}")
        assert info[i] == (0, 0)
        if n == 0 or k == 0:
            continue
        Xref, st = oracle.ls(As[i], Bs[i])
        assert st == 0
        assert oracle.rel_fro(Xs[i], Xref) <= 1e-11, (m, n, k)
        assert oracle.ls_eta(As[i], Xs[i], Bs[i]) <= 1e-14
        Xp, ip = caqr.ls_solve(caqr.fortran(As[i]), caqr.fortran(Bs[i]))
        torch.cuda.synchronize()
        assert ip.status == 0
        assert oracle.rel_fro(Xs[i], Xp.cpu().numpy()) <= 1e-12


@pytest.mark.parametrize("leaf_rows,lpw,arity", [(64, 1, 4), (128, 2, 2), (256, 4, 4), (64, 4, 2)])
def test_batched_ls_plans(leaf_rows, lpw, arity):
    require_gpu()
    mix = MIX[:7]
    As, Bs, Xs, info = run(mix, 8200 + leaf_rows + lpw, leaf_rows=leaf_rows, leaves_per_wg=lpw, arity=arity)
    for i, (m, n, k) in enumerate(mix):
        assert info[i] == (0, 0)
        Xref, _ = oracle.ls(As[i], Bs[i])
        assert oracle.rel_fro(Xs[i], Xref) <= 1e-11, (m, n, k, leaf_rows, lpw, arity)


def test_batched_ls_conditioned_consistent():
    """b = A x_true with kappa(A) up to 1e6: x_true recovered within kappa u."""
    require_gpu()
    rng = np.random.default_rng(83)
    As, Bs, xs = [], [], []
    for kappa, (m, n) in zip((1e2, 1e4, 1e6), ((3000, 40), (10000, 64), (700, 20))):
        U = np.linalg.qr(rng.standard_normal((m, n)))[0]
        V = np.linalg.qr(rng.standard_normal((n, n)))[0]
        A = (U * inputs.geometric_singular_values(n, kappa)) @ V.T
        x = rng.standard_normal(n)
        As.append(A)
        Bs.append((A @ x)[:, None])
        xs.append((x, kappa))
    Xs, info = caqr.ls_solve_batched([caqr.fortran(a) for a in As], [caqr.fortran(b) for b in Bs])
    torch.cuda.synchronize()
    for X, (x, kappa), st, A in zip(Xs, xs, info, As):
        assert st == (0, 0)
        n = len(x)
        assert np.linalg.norm(X.cpu().numpy()[:, 0] - x) / np.linalg.norm(x) <= 50 * kappa * 2.0 ** -53 * n


def test_batched_ls_statuses():
    """A zero column (SINGULAR at its index) and an infinite entry (NONFINITE)
    in the same batch as regular problems, which are unaffected."""
    require_gpu()
    A1 = inputs.gaussian(500, 20, 8300)
    A1[:, 5] = 0.0
    A2 = inputs.gaussian(600, 16, 8301)
    A2[3, 3] = np.inf
    A3 = inputs.gaussian(800, 24, 8302)
    B = [inputs.gaussian(a.shape[0], 1, 8310 + i) for i, a in enumerate((A1, A2, A3))]
    Xs, info = caqr.ls_solve_batched([caqr.fortran(a) for a in (A1, A2, A3)], [caqr.fortran(b) for b in B])
    torch.cuda.synchronize()
    assert info[0] == (5, 5)
    assert info[1][0] == 6
    assert info[2] == (0, 0)
    Xref, _ = oracle.ls(A3, B[2])
    assert oracle.rel_fro(Xs[2].cpu().numpy(), Xref) <= 1e-11
