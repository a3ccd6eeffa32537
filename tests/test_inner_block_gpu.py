"""Per-level block sizes (paper, Section 3.1, item 1(a)): each leaf and each
stacked elimination of a panel of width b factored in inner blocks of 16 or 32
columns, every finished block applied to the columns right of it at once.

The reflectors are those of the unblocked factorization up to rounding, so the
bars are the same as for every other factorization: R within 1e-11 of the
oracle, the invariants at 1e-13, and the exact identities of the method
(grouping of leaves into workgroups, power-of-two scaling, exact zeros)."""
import numpy as np
import pytest

import oracle
from paper_1303_5837_amd import inputs
from tests._gpu import banner, caqr_gpu, factored, q_thin, require_gpu, tsqr_gpu

pytestmark = pytest.mark.gpu

TOL_R = 1e-11
TOL_INV = 1e-13

TSQR_CASES = [
    # (m, n, leaf_rows, leaves_per_wg, inner_block)
    (4096, 64, 256, 0, 16),
    (4096, 64, 256, 0, 32),
    (4096, 32, 256, 1, 16),
    (1000, 20, 256, 0, 16),   # second block holds 4 columns
    (3001, 50, 64, 2, 32),    # second block holds 18 columns, ragged last leaf
    (2600, 48, 128, 4, 16),   # last leaf holds 40 rows < n
    (2600, 48, 128, 4, 32),
    (300, 64, 64, 4, 32),
    (100, 64, 256, 0, 16),    # one leaf shorter than leaf_rows
    (40000, 17, 256, 1, 16),  # 157 workgroups: tree levels launched one by one
    (40000, 40, 128, 4, 32),  # ticket climbs over 79 workgroups
    (5000, 16, 256, 0, 16),   # block as wide as the panel: no inner blocking
    (33000, 64, 128, 2, 32),  # 128-row leaves: w and z of the block update through LDS
    (33000, 64, 256, 1, 16),
]


@pytest.mark.parametrize("m,n,h,lpw,ib", TSQR_CASES)
def test_tsqr_matches_oracle(m, n, h, lpw, ib):
    require_gpu()
    banner(f"inner-block tsqr parity m={m} n={n} leaf_rows={h} lpw={lpw} inner_block={ib}")
    A = inputs.gaussian(m, n, 3000 + m + n + ib)
    F, R = tsqr_gpu(A, leaf_rows=h, leaves_per_wg=lpw, inner_block=ib)
    assert F.info().inner_block == ib
    Rref = oracle.qr_r(A)
    assert np.all(np.diag(R) >= 0)
    assert oracle.rel_fro(R, Rref) <= TOL_R
    R0 = tsqr_gpu(A, leaf_rows=h, leaves_per_wg=lpw)[1]
    assert oracle.rel_fro(R, R0) <= TOL_INV
    if m * n <= 200000:
        Q = q_thin(F)
        assert oracle.factorization_error(A, Q, R) <= TOL_INV
        assert oracle.orthogonality_error(Q) <= TOL_INV


CAQR_CASES = [
    # (m, n, nb, inner_block)
    (1000, 700, 64, 16),
    (1000, 700, 64, 32),
    (777, 200, 32, 16),
    (700, 90, 17, 16),     # panels of 17 columns: a one-column second block
    (3000, 1000, 64, 32),
    (1200, 600, 64, 32),   # with 128-row leaves (see the test)
]


@pytest.mark.parametrize("m,n,nb,ib", CAQR_CASES)
def test_caqr_matches_oracle(m, n, nb, ib):
    require_gpu()
    banner(f"inner-block caqr parity m={m} n={n} nb={nb} inner_block={ib}")
    A = inputs.gaussian(m, n, 4000 + m + n + ib)
    F, R = caqr_gpu(A, nb=nb, inner_block=ib, leaf_rows=128 if (m, n) == (1200, 600) else 0)
    oracle.set_threads(16)
    Rref = oracle.qr_r(A)
    assert np.all(np.diag(R) >= 0)
    assert oracle.rel_fro(R, Rref) <= TOL_R


def test_caqr_invariants():
    require_gpu()
    banner("inner-block caqr 1500x1100 invariants")
    A = inputs.gaussian(1500, 1100, 91)
    for ib in (16, 32):
        F, R = caqr_gpu(A, inner_block=ib)
        Q = q_thin(F)
        assert oracle.factorization_error(A, Q, R) <= TOL_INV
        assert oracle.orthogonality_error(Q) <= TOL_INV


def test_grouping_and_determinism():
    """leaves_per_wg only moves tree levels between a workgroup and the device,
    with or without inner blocks: bitwise equal; repeated runs bitwise equal."""
    require_gpu()
    for m, seed in ((9000, 177), (40000, 176)):
        A = inputs.gaussian(m, 40, seed)
        outs = [factored(tsqr_gpu(A, leaf_rows=128, leaves_per_wg=lpw, inner_block=32)[0]) for lpw in (1, 2, 4)]
        assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2]), m
    A = inputs.gaussian(20000, 64, 178)
    a = factored(tsqr_gpu(A, inner_block=16)[0])
    for _ in range(2):
        assert np.array_equal(factored(tsqr_gpu(A, inner_block=16)[0]), a)


def test_power_of_two_scaling_is_exact():
    """Every product in a block update has exactly one scaled factor, so
    R(2^k A) = 2^k R(A) holds bitwise, on the rescaled norm path too."""
    require_gpu()
    A = inputs.gaussian(5000, 48, 180)
    for ib in (16, 32):
        R = tsqr_gpu(A, inner_block=ib)[1]
        for k in (-3, 5, 200, -1000, 1000):
            Rk = tsqr_gpu(np.ldexp(A, k), inner_block=ib)[1]
            assert np.array_equal(Rk, np.ldexp(R, k)), (ib, k)


def test_exact_zeros():
    """Upper triangular input with mixed signs: every tau is 0, the block
    updates add exact zeros, and R = D A(0:n) bitwise; the zero matrix gives
    R = 0 and Q = I."""
    require_gpu()
    rng = np.random.default_rng(181)
    n = 40
    A = np.zeros((2000, n))
    A[:n] = np.triu(rng.standard_normal((n, n)))
    d = np.where(np.diag(A[:n]) < 0, -1.0, 1.0)
    for ib in (16, 32):
        R = tsqr_gpu(A, inner_block=ib)[1]
        assert np.array_equal(R, d[:, None] * A[:n]), ib
        F, R = tsqr_gpu(np.zeros((777, 33)), inner_block=ib)
        assert np.all(R == 0)
        assert np.array_equal(q_thin(F), np.eye(777, 33))
