"""CAQR (panel loop with tree panels and trailing updates) on the GPU vs the oracle."""
import os

import numpy as np
import pytest
import torch

import oracle
from paper_1303_5837_amd import caqr, inputs
from tests._gpu import banner, caqr_gpu, factored, q_thin, require_gpu, tsqr_gpu

pytestmark = pytest.mark.gpu

TOL_R = 1e-11
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

CASES = [
    # (m, n, nb, leaf_rows)
    (512, 384, 64, 0),
    (1000, 700, 64, 0),    # ragged leaves and panels
    (1024, 1024, 64, 0),
    (777, 200, 32, 0),
    (1200, 130, 64, 0),    # last panel of width 2
    (4096, 300, 64, 128),
    (3000, 3000, 64, 64),
    (2048, 2048, 64, 0),
    (700, 90, 17, 0),      # odd panel width
]


@pytest.mark.parametrize("arity", [4, 2])
@pytest.mark.parametrize("m,n,nb,h", CASES)
def test_r_matches_oracle(m, n, nb, h, arity):
    require_gpu()
    banner(f"caqr parity m={m} n={n} nb={nb} leaf_rows={h} arity={arity}")
    A = inputs.gaussian(m, n, 2000 + m + n)
    F, R = caqr_gpu(A, nb=nb, leaf_rows=h, arity=arity)
    assert F.info().arity == arity
    oracle.set_threads(16)
    Rref = oracle.qr_r(A)
    assert np.all(np.diag(R) >= 0)
    assert oracle.rel_fro(R, Rref) <= TOL_R


@pytest.mark.parametrize("arity", [4, 2])
def test_invariants(arity):
    require_gpu()
    A = inputs.gaussian(1500, 1100, 91)
    F, R = caqr_gpu(A, arity=arity)
    Q = q_thin(F)
    assert oracle.factorization_error(A, Q, R) <= 1e-13
    assert oracle.orthogonality_error(Q) <= 1e-13


@pytest.mark.parametrize("m,n", [(3000, 700), (2850, 700), (2048, 640)])
def test_resident_passes_match_per_tile_passes(m, n):
    """The wide update's leaf pass and node levels run with the reflectors of
    each leaf (node) resident in LDS where C allows 16-byte accesses (even
    leading dimension), else one workgroup per leaf (node) and 32-column tile;
    both form the same products in the same order, so the factorizations are
    bitwise equal (partial last leaf, a node member with fewer than 64 rows
    (m = 2850), nodes of 3 members and partial last tiles included; and leaf
    passes with no edge job at all (2048 x 640: whole leaves and whole
    128-column tiles in its first calls))."""
    require_gpu()
    banner(f"caqr: resident passes vs per-tile passes, {m} x {n}")
    A = inputs.gaussian(m, n, 95)
    F1, _ = caqr_gpu(A)
    P = torch.zeros((n, m + 1), dtype=torch.float64, device="cuda").t()[:m, :]  # leading dimension m + 1
    P.copy_(torch.as_tensor(A, device="cuda"))
    F2 = caqr.caqr(P)
    torch.cuda.synchronize()
    assert np.array_equal(factored(F1), P.cpu().numpy())
    F2.close()


@pytest.mark.parametrize("m,k", [(200, 300), (1024, 256), (3000, 330)])
def test_resident_apply_qt_matches_per_tile(m, k):
    """Q^T of an m x 64 TSQR applied to C = [A, G] (m x k): the leaf pass with
    the reflectors resident in LDS (even leading dimension) and the per-tile
    leaf kernel (odd) agree bitwise, on a leaf pass of edge jobs only (m = 200,
    one short leaf), one with none (1024 x 256: whole leaves and tiles) and one
    with both; Q^T A is [R; 0] and Q Q^T C returns C."""
    require_gpu()
    banner(f"apply_q: resident leaf pass vs per-tile, {m} x 64 applied to {m} x {k}")
    A = inputs.gaussian(m, 64, 96)
    F, R = tsqr_gpu(A)
    C0 = np.concatenate([A, np.random.default_rng(7).standard_normal((m, k - 64))], axis=1)
    C1 = caqr.fortran(C0)
    C2 = torch.zeros((k, m + 1), dtype=torch.float64, device="cuda").t()[:m, :]  # leading dimension m + 1
    C2.copy_(torch.as_tensor(C0, device="cuda"))
    F.apply_q(C1, caqr.OP_T)
    F.apply_q(C2, caqr.OP_T)
    torch.cuda.synchronize()
    X = C1.cpu().numpy()
    assert np.array_equal(X, C2.cpu().numpy())
    assert oracle.rel_fro(X[:64, :64], R) <= 1e-13
    assert np.abs(X[64:, :64]).max() <= 1e-13 * np.linalg.norm(A)
    F.apply_q(C1, caqr.OP_N)
    torch.cuda.synchronize()
    assert oracle.rel_fro(C1.cpu().numpy(), C0) <= 1e-14
    F.close()


def test_determinism():
    require_gpu()
    A = inputs.gaussian(2000, 1500, 92)
    a = factored(caqr_gpu(A)[0])
    assert np.array_equal(factored(caqr_gpu(A)[0]), a)


# Panels of 128 or more workgroups (m_s >= 128 leaves of 256 rows) finish their
# trees with one launch per level, and the next panel's columns are updated
# level by level too: the path of the tall least-squares shapes.
TALL = [(40000, 200), (65536, 1024)]


@pytest.mark.parametrize("arity", [4, 2])
@pytest.mark.parametrize("m,n", TALL)
def test_tall_caqr_level_path(m, n, arity):
    """R against the oracle, Q_thin^T C (unique for full-rank A) against the
    oracle's, the round trip Q (Q^T C) = C, and Q^T A = [R; 0]."""
    require_gpu()
    banner(f"tall caqr parity m={m} n={n} arity={arity}")
    A = inputs.gaussian(m, n, 2100 + n)
    dA0 = caqr.fortran(A)
    F, R = caqr_gpu(A, arity=arity)
    assert F.info().leaves_panel0 >= 128
    oracle.set_threads(16)
    f = oracle.qr(A)
    assert np.all(np.diag(R) >= 0)
    assert oracle.rel_fro(R, f.R) <= TOL_R
    C = inputs.gaussian(m, 8, 2200 + n)
    dC = caqr.fortran(C)
    F.apply_q(dC, caqr.OP_T)
    torch.cuda.synchronize()
    QtC = dC.cpu().numpy()
    assert oracle.rel_fro(QtC[:n], f.apply_qt(C)[:n]) <= TOL_R
    F.apply_q(dC, caqr.OP_N)
    torch.cuda.synchronize()
    assert oracle.rel_fro(dC.cpu().numpy(), C) <= 1e-14
    F.apply_q(dA0, caqr.OP_T)  # Q^T A: R on top, zero below
    torch.cuda.synchronize()
    QtA = dA0.cpu().numpy()
    nrm = np.linalg.norm(A)
    assert np.linalg.norm(QtA[:n] - R) / nrm <= 1e-13
    assert np.linalg.norm(QtA[n:]) / nrm <= 1e-13


def test_square_8192_full():
    """The square configuration at full size: every entry of R against the
    oracle run in the test, plus the stored oracle sample
    (tests/golden/make_golden.py, oracle only) and the Gram identity
    R^T R = A^T A on sampled entries."""
    require_gpu()
    banner("caqr 8192x8192 full-size parity (oracle in the test)")
    A = inputs.gaussian(8192, 8192, inputs.SEEDS["caqr_8192sq"])
    F, R = caqr_gpu(A)
    del F
    oracle.set_threads(16)
    Rref = oracle.qr_r(A)
    assert np.all(np.diag(R) >= 0)
    assert oracle.rel_fro(R, Rref) <= TOL_R
    col = np.linalg.norm(R - Rref, axis=0) / np.linalg.norm(Rref, axis=0)
    banner(f"  normwise {oracle.rel_fro(R, Rref):.2e}, worst column {col.max():.2e}")
    assert col.max() <= TOL_R
    g = np.load(os.path.join(GOLDEN, "caqr_8192_r_sample.npz"))
    ii, jj, ref = g["i"], g["j"], g["r"]
    assert np.linalg.norm(R[ii, jj] - ref) / np.linalg.norm(ref) <= TOL_R
    assert np.linalg.norm(np.diag(R) - g["diag"]) / np.linalg.norm(g["diag"]) <= TOL_R
    rng = np.random.default_rng(93)
    pi = rng.integers(0, 8192, 200)
    pj = rng.integers(0, 8192, 200)
    gram = np.einsum("ij,ij->j", A[:, pi], A[:, pj])
    rtr = np.einsum("ij,ij->j", R[:, pi], R[:, pj])
    norms = np.linalg.norm(A[:, pi], axis=0) * np.linalg.norm(A[:, pj], axis=0)
    assert np.max(np.abs(rtr - gram) / norms) <= 1e-13
