"""TSQR (one panel, reduction tree of arity 2 or 4) on the GPU vs the oracle.

Bars: ||R - R_oracle||_F / ||R_oracle||_F <= 1e-11 (FP64), ||A - QR||/||A|| and
||I - Q^T Q|| <= 1e-13, and the exact identities of the method (tree shape and
workgroup grouping do not change R; R(2^k A) = 2^k R(A) bitwise; bitwise
determinism)."""
import numpy as np
import pytest

import oracle
from paper_1303_5837_amd import inputs
from tests import _exact
from tests._gpu import banner, factored, q_thin, require_gpu, tsqr_gpu

pytestmark = pytest.mark.gpu

TOL_R = 1e-11
TOL_INV = 1e-13

CASES = [
    # (m, n, leaf_rows, leaves_per_wg)
    (4096, 32, 256, 0),   # 16 leaves of 256 rows, binary tree of 4 levels
    (4096, 32, 256, 1),
    (4096, 32, 64, 2),
    (1000, 7, 256, 4),    # ragged last leaf
    (2600, 48, 128, 4),   # last leaf holds 40 rows < n
    (257, 33, 256, 0),    # last leaf holds 1 row
    (300, 64, 64, 4),
    (64, 64, 64, 1),      # one square leaf
    (100, 64, 256, 0),    # one leaf shorter than leaf_rows
    (5000, 1, 256, 0),
    (1, 1, 256, 0),
    (40000, 17, 256, 4),  # 157 leaves, several device levels
    (40000, 17, 256, 1),  # 157 workgroups: tree finished by one launch per level
    (33000, 64, 128, 2),
]


@pytest.mark.parametrize("m,n,h,lpw", CASES)
def test_r_matches_oracle(m, n, h, lpw):
    require_gpu()
    banner(f"tsqr parity m={m} n={n} leaf_rows={h} lpw={lpw}")
    A = inputs.gaussian(m, n, 1000 + m + n)
    F, R = tsqr_gpu(A, leaf_rows=h, leaves_per_wg=lpw)
    Rref = oracle.qr_r(A)
    assert np.all(np.diag(R) >= 0)
    assert oracle.rel_fro(R, Rref) <= TOL_R
    col = np.linalg.norm(R - Rref, axis=0) / np.linalg.norm(Rref, axis=0)
    assert col.max() <= TOL_R
    d = F.signs()
    assert set(np.unique(d)) <= {-1.0, 1.0}


def test_config0_invariants_and_apply_q():
    require_gpu()
    banner("tsqr 4096x32 invariants")
    A = inputs.gaussian(4096, 32, inputs.SEEDS["tsqr_4096x32"])
    F, R = tsqr_gpu(A, arity=2)  # this configuration's binary tree over 16 leaves
    info = F.info()
    assert info.leaves_panel0 == 16 and info.depth_panel0 == 4 and info.arity == 2
    Q = q_thin(F)
    assert oracle.factorization_error(A, Q, R) <= TOL_INV
    assert oracle.orthogonality_error(Q) <= TOL_INV
    # Q^T then Q is the identity
    import torch

    from paper_1303_5837_amd import caqr

    C0 = np.random.default_rng(5).standard_normal((4096, 9))
    C = caqr.fortran(C0)
    F.apply_q(C, caqr.OP_T)
    QtC = C.cpu().numpy()
    assert oracle.rel_fro(QtC[:32], Q.T @ C0) <= 1e-13
    F.apply_q(C, caqr.OP_N)
    torch.cuda.synchronize()
    assert oracle.rel_fro(C.cpu().numpy(), C0) <= 1e-14
    # (Q^T A)(0:n) = R
    Ca = caqr.fortran(A)
    F.apply_q(Ca, caqr.OP_T)
    QtA = Ca.cpu().numpy()
    assert oracle.rel_fro(np.triu(QtA[:32]), R) <= 1e-13
    assert np.abs(QtA[32:]).max() <= 1e-12 * np.abs(A).max() * 64


@pytest.mark.parametrize("arity,lpws", [(2, (1, 2, 4)), (4, (1, 4))])
def test_grouping_does_not_change_anything(arity, lpws):
    """leaves_per_wg only moves tree levels between a workgroup and the device: bitwise equal.
    At 40000 rows (313 leaves of 128) one and two leaves per workgroup finish the tree by one
    launch per level, four by ticket climbs: the two device-level schemes agree bitwise too."""
    require_gpu()
    for m, seed in ((9000, 77), (40000, 76)):
        A = inputs.gaussian(m, 40, seed)
        outs = []
        for lpw in lpws:
            F, R = tsqr_gpu(A, leaf_rows=128, leaves_per_wg=lpw, arity=arity)
            assert F.info().arity == arity
            outs.append(factored(F))
        for o in outs[1:]:
            assert np.array_equal(outs[0], o), (m, arity)


# (m, n, leaf_rows, leaves_per_wg): leaf counts that are and are not powers of
# four, groups with 2 and 3 members at the end of a level, one leaf, ticket
# climbs and level launches (128 or more workgroups)
ARITY_CASES = [(4096, 32, 256, 1), (1000, 7, 256, 1), (1280, 20, 256, 1), (1536, 64, 256, 1), (2600, 48, 128, 4),
               (300, 64, 64, 1), (257, 33, 256, 4), (100, 64, 256, 1), (40000, 17, 256, 4), (40000, 17, 256, 1),
               (70000, 64, 64, 1), (33000, 64, 128, 4)]


@pytest.mark.parametrize("m,n,h,lpw", ARITY_CASES)
def test_arity4_against_oracle_and_binary(m, n, h, lpw):
    """Arity-4 trees: R against the oracle, against the binary tree's R (the
    same R of a full-rank A: tree independence), Q's invariants and the Q^T / Q
    round trip."""
    require_gpu()
    banner(f"arity-4 tsqr m={m} n={n} leaf_rows={h} lpw={lpw}")
    A = inputs.gaussian(m, n, 1500 + m + n)
    F, R = tsqr_gpu(A, leaf_rows=h, leaves_per_wg=lpw, arity=4)
    assert F.info().arity == 4
    L = -(-m // h)
    depth = 0
    while 4 ** depth < L:
        depth += 1
    assert F.info().depth_panel0 == depth
    Rref = oracle.qr_r(A)
    assert np.all(np.diag(R) >= 0)
    assert oracle.rel_fro(R, Rref) <= TOL_R
    R2 = tsqr_gpu(A, leaf_rows=h, leaves_per_wg=1, arity=2)[1]
    assert oracle.rel_fro(R, R2) <= TOL_INV
    if m * n <= 400000:
        Q = q_thin(F)
        assert oracle.factorization_error(A, Q, R) <= TOL_INV
        assert oracle.orthogonality_error(Q) <= TOL_INV
    import torch

    from paper_1303_5837_amd import caqr

    C0 = np.random.default_rng(6).standard_normal((m, 3))
    C = caqr.fortran(C0)
    F.apply_q(C, caqr.OP_T)
    F.apply_q(C, caqr.OP_N)
    torch.cuda.synchronize()
    assert oracle.rel_fro(C.cpu().numpy(), C0) <= 1e-14


def test_leaf_height_independence():
    require_gpu()
    A = inputs.gaussian(12345, 50, 78)
    Rs = [tsqr_gpu(A, leaf_rows=h, arity=k)[1] for h in (64, 128, 256) for k in (2, 4)]
    for R in Rs[1:]:
        assert oracle.rel_fro(R, Rs[0]) <= 1e-13


def test_determinism():
    require_gpu()
    A = inputs.gaussian(70000, 64, 79)
    a = factored(tsqr_gpu(A)[0])
    for _ in range(3):
        assert np.array_equal(factored(tsqr_gpu(A)[0]), a)


def test_power_of_two_scaling_is_exact():
    require_gpu()
    A = inputs.gaussian(5000, 24, 80)
    R = tsqr_gpu(A)[1]
    for k in (-3, 5, 200, -200):
        Rk = tsqr_gpu(np.ldexp(A, k))[1]
        assert np.array_equal(Rk, np.ldexp(R, k)), k


def test_extreme_scaling_rescue_path():
    """Entries near the underflow/overflow limits: the scaled norm path keeps R exact up to rounding."""
    require_gpu()
    A = inputs.gaussian(3000, 16, 81)
    R0 = tsqr_gpu(A)[1]
    for k in (-1000, 1000):  # squares under/overflow, entries and products do not
        As = np.ldexp(A, k)
        R = tsqr_gpu(As)[1]
        Rref = oracle.qr_r(As)
        assert np.all(np.isfinite(R))
        assert oracle.rel_fro(np.ldexp(R, -k), np.ldexp(Rref, -k)) <= 1e-11, k
        # the rescaled sums keep the unscaled summation order: still exact
        assert np.array_equal(R, np.ldexp(R0, k)), k
    # subnormal entries keep ~14 significant bits and the updates round at the
    # subnormal spacing, so only finiteness and agreement to 1e-2 are meaningful
    As = np.ldexp(A, -1060)
    R = tsqr_gpu(As)[1]
    Rref = oracle.qr_r(As)
    assert np.all(np.isfinite(R)) and np.all(np.isfinite(Rref))
    assert oracle.rel_fro(np.ldexp(R, 1060), np.ldexp(Rref, 1060)) <= 1e-2


def test_dyadic_rows_spread_over_leaves():
    require_gpu()
    for (m, n) in [(1024, 8), (1024, 32), (4096, 64)]:
        A, R0 = _exact.dyadic_case(m, n, seed=m + n)
        R = tsqr_gpu(A)[1]
        assert oracle.rel_fro(R, R0) <= 64 * n * 2.0 ** -53


def test_structured_inputs():
    require_gpu()
    rng = np.random.default_rng(82)
    # upper triangular with mixed signs: R = D A(0:n) bitwise
    n = 40
    A = np.zeros((2000, n))
    A[:n] = np.triu(rng.standard_normal((n, n)))
    R = tsqr_gpu(A)[1]
    d = np.where(np.diag(A[:n]) < 0, -1.0, 1.0)
    assert np.array_equal(R, d[:, None] * A[:n])
    # zero matrix
    Z = np.zeros((777, 9))
    F, R = tsqr_gpu(Z)
    assert np.all(R == 0)
    assert np.array_equal(q_thin(F), np.eye(777, 9))
    # rank deficient: a zero column and a repeated column
    B = rng.standard_normal((1500, 12))
    B[:, 3] = 0.0
    B[:, 7] = B[:, 2]
    F, R = tsqr_gpu(B)
    assert abs(R[3, 3]) == 0.0 and abs(R[7, 7]) <= 1e-12 * abs(R[2, 2])
    Q = q_thin(F)
    assert oracle.factorization_error(B, Q, R) <= TOL_INV
    # row permutation invariance: R(PA) = R(A)
    C = inputs.gaussian(6000, 30, 83)
    R1 = tsqr_gpu(C)[1]
    R2 = tsqr_gpu(C[rng.permutation(6000)])[1]
    assert oracle.rel_fro(R2, R1) <= 1e-13


def test_nan_propagates_without_error():
    require_gpu()
    A = inputs.gaussian(2048, 8, 84)
    A[1000, 3] = np.nan
    R = tsqr_gpu(A)[1]
    assert np.isnan(R[3:, 3:]).any() or np.isnan(R).any()


def test_tall_1m_by_64():
    """The tall configuration at full size (1,048,576 x 64), default tree."""
    require_gpu()
    banner("tsqr 1048576x64 full-size parity")
    A = inputs.gaussian(1 << 20, 64, inputs.SEEDS["tsqr_1Mx64"])
    F, R = tsqr_gpu(A)
    info = F.info()
    assert info.leaves_panel0 == 4096
    oracle.set_threads(16)
    Rref = oracle.qr_r(A)
    assert oracle.rel_fro(R, Rref) <= TOL_R
    # property at any size: R^T R = A^T A
    G = A.T @ A
    assert oracle.rel_fro(R.T @ R, G) <= 1e-13
