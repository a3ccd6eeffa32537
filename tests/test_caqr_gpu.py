"""CAQR (panel loop with tree panels and trailing updates) on the GPU vs the oracle."""
import os

import numpy as np
import pytest

import oracle
from paper_1303_5837_amd import inputs
from tests._gpu import banner, caqr_gpu, factored, q_thin, require_gpu

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


@pytest.mark.parametrize("m,n,nb,h", CASES)
def test_r_matches_oracle(m, n, nb, h):
    require_gpu()
    banner(f"caqr parity m={m} n={n} nb={nb} leaf_rows={h}")
    A = inputs.gaussian(m, n, 2000 + m + n)
    F, R = caqr_gpu(A, nb=nb, leaf_rows=h)
    oracle.set_threads(16)
    Rref = oracle.qr_r(A)
    assert np.all(np.diag(R) >= 0)
    assert oracle.rel_fro(R, Rref) <= TOL_R


def test_invariants():
    require_gpu()
    A = inputs.gaussian(1500, 1100, 91)
    F, R = caqr_gpu(A)
    Q = q_thin(F)
    assert oracle.factorization_error(A, Q, R) <= 1e-13
    assert oracle.orthogonality_error(Q) <= 1e-13


def test_determinism():
    require_gpu()
    A = inputs.gaussian(2000, 1500, 92)
    a = factored(caqr_gpu(A)[0])
    assert np.array_equal(factored(caqr_gpu(A)[0]), a)


def test_square_8192_sampled():
    """The square configuration at full size: sampled entries of R against stored
    oracle values (tests/golden/make_golden.py, oracle only) and the Gram identity
    R^T R = A^T A on sampled entries."""
    require_gpu()
    banner("caqr 8192x8192 full-size sampled parity")
    path = os.path.join(GOLDEN, "caqr_8192_r_sample.npz")
    g = np.load(path)
    A = inputs.gaussian(8192, 8192, inputs.SEEDS["caqr_8192sq"])
    F, R = caqr_gpu(A)
    ii, jj, ref = g["i"], g["j"], g["r"]
    got = R[ii, jj]
    scale = np.linalg.norm(g["diag"])
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= TOL_R
    assert np.linalg.norm(np.diag(R) - g["diag"]) / scale <= TOL_R
    rng = np.random.default_rng(93)
    pi = rng.integers(0, 8192, 200)
    pj = rng.integers(0, 8192, 200)
    gram = np.einsum("ij,ij->j", A[:, pi], A[:, pj])
    rtr = np.einsum("ij,ij->j", R[:, pi], R[:, pj])
    norms = np.linalg.norm(A[:, pi], axis=0) * np.linalg.norm(A[:, pj], axis=0)
    assert np.max(np.abs(rtr - gram) / norms) <= 1e-13
