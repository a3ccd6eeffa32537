"""Single-precision batched TSQR (float storage and arithmetic, the same steps as
the double-precision path).  Inputs are the double draws rounded to float; the
oracle factors those values in double.  Bounds for single precision: R within
1e-5 of the oracle, normwise, and R^T R = A^T A within 1e-5 (about 170 units of
float rounding).  Each problem's result does not depend on the rest of the
batch (bitwise), and power-of-two scaling is exact (bitwise), also where the
sums of squares underflow or overflow in float."""
import numpy as np
import pytest
import torch

import oracle
from paper_1303_5837_amd import caqr, inputs
from tests._gpu import banner, require_gpu

pytestmark = pytest.mark.gpu

TOL32 = 1e-5

SIZES = [(1, 1), (7, 5), (64, 64), (100, 8), (255, 16), (256, 17), (257, 32), (300, 1), (511, 33),
         (700, 64), (1000, 40), (1024, 64), (1500, 8), (2049, 16), (3000, 32), (4096, 64), (5000, 3),
         (6000, 64), (129, 64)]


def make32(sizes, seed):
    hosts = [inputs.gaussian(m, n, seed + i, dtype=np.float32) for i, (m, n) in enumerate(sizes)]
    devs = [caqr.fortran(a, dtype=torch.float32) for a in hosts]
    return hosts, devs


def gram_residual(A, R):
    A = A.astype(np.float64)
    R = R.astype(np.float64)
    G = A.T @ A
    return np.linalg.norm(R.T @ R - G) / np.linalg.norm(G)


def check32(sizes, seed, **plan):
    hosts, devs = make32(sizes, seed)
    B = caqr.tsqr_batched(devs, **plan)
    torch.cuda.synchronize()
    outs = []
    for i, (m, n) in enumerate(sizes):
        banner(f"f32 batched problem {i}: m={m} n={n} plan={B.plan(i)}")
        got = devs[i].cpu().numpy()
        outs.append(got)
        R = np.triu(got[:n, :n]).astype(np.float64)
        assert np.all(np.diag(R) >= 0)
        assert oracle.rel_fro(R, oracle.qr_r(hosts[i].astype(np.float64))) <= TOL32, (m, n)
        assert gram_residual(hosts[i], R) <= TOL32, (m, n)
        d = B.signs(i)
        assert np.all(np.abs(d) == 1.0)
    B.close()
    return hosts, outs


def test_f32_fixed_plan_against_oracle():
    require_gpu()
    oracle.set_threads(16)
    check32(SIZES, 700, leaf_rows=256, leaves_per_wg=4)


@pytest.mark.parametrize("leaf_rows,lpw,arity", [(64, 1, 4), (128, 2, 2), (64, 4, 4), (256, 1, 2), (128, 4, 2)])
def test_f32_other_plans(leaf_rows, lpw, arity):
    require_gpu()
    check32(SIZES[:12], 800 + leaf_rows + lpw, leaf_rows=leaf_rows, leaves_per_wg=lpw, arity=arity)


def test_f32_alone_equals_in_batch():
    """A problem factored alone and inside a mixed batch: bitwise the same."""
    require_gpu()
    sizes = SIZES[:10]
    hosts, outs = check32(sizes, 900)
    for i in (1, 4, 9):
        d = caqr.fortran(hosts[i], dtype=torch.float32)
        B = caqr.tsqr_batched([d])
        torch.cuda.synchronize()
        assert np.array_equal(d.cpu().numpy(), outs[i]), sizes[i]
        B.close()


@pytest.mark.parametrize("k", [-70, -40, 40, 70])
def test_f32_power_of_two_scaling_is_exact(k):
    """R(2^k A) = 2^k R(A) bitwise; at k = -70 the float sums of squares are
    subnormal, at k = 70 they overflow, so the scaled recomputation is taken."""
    require_gpu()
    m, n = 1000, 24
    A = inputs.gaussian(m, n, 950, dtype=np.float32)
    d0 = caqr.fortran(A, dtype=torch.float32)
    d1 = caqr.fortran(np.ldexp(A, k).astype(np.float32), dtype=torch.float32)
    B = caqr.tsqr_batched([d0, d1], leaf_rows=128, leaves_per_wg=2)
    torch.cuda.synchronize()
    R0 = np.triu(d0.cpu().numpy()[:n, :n])
    R1 = np.triu(d1.cpu().numpy()[:n, :n])
    assert np.array_equal(np.ldexp(R0, k).astype(np.float32), R1)
    B.close()


def test_f32_zero_and_structured_columns():
    """Zero columns (tau = 0, a zero column of R) and an upper-triangular input
    (R = D A bitwise)."""
    require_gpu()
    m, n = 600, 20
    A = inputs.gaussian(m, n, 960, dtype=np.float32)
    A[:, 3] = 0.0
    A[:, 11] = 0.0
    U = np.zeros((300, 16), dtype=np.float32, order="F")
    U[:16, :16] = np.triu(inputs.gaussian(16, 16, 961, dtype=np.float32))
    dA = caqr.fortran(A, dtype=torch.float32)
    dU = caqr.fortran(U, dtype=torch.float32)
    B = caqr.tsqr_batched([dA, dU], leaf_rows=64, leaves_per_wg=2)
    torch.cuda.synchronize()
    R = np.triu(dA.cpu().numpy()[:n, :n]).astype(np.float64)
    # rank deficient: only R's zero columns and R^T R are unique
    assert np.all(R[:, 3] == 0.0) and np.all(R[:, 11] == 0.0)
    assert np.all(np.diag(R) >= 0)
    assert gram_residual(A, R) <= TOL32
    RU = np.triu(dU.cpu().numpy()[:16, :16])
    D = np.where(np.diag(U[:16, :16]) < 0, -1.0, 1.0).astype(np.float32)
    assert np.array_equal(RU, D[:, None] * U[:16, :16])
    B.close()


def test_f32_tuner_and_default_plans():
    require_gpu()
    caqr.tune_batched(dtype=torch.float32)
    sizes = [(300, 8), (5000, 16), (40000, 64), (70000, 32), (100, 64)]
    for m, n in sizes:
        hr, lpw, ar = caqr.batch_plan_for(m, n, dtype=torch.float32)
        assert hr in (64, 128, 256) and (ar, lpw) in ((2, 1), (2, 2), (2, 4), (4, 1), (4, 4))
    hosts, devs = make32(sizes, 980)
    B = caqr.tsqr_batched(devs)
    torch.cuda.synchronize()
    for i, (m, n) in enumerate(sizes):
        assert B.plan(i) == caqr.batch_plan_for(m, n, dtype=torch.float32)
        R = np.triu(devs[i].cpu().numpy()[:n, :n]).astype(np.float64)
        assert gram_residual(hosts[i], R) <= TOL32
    B.close()


def test_f32_full_uneven_batch():
    """The uneven 2000-problem batch in float (the double draws rounded), in the
    plan the benchmark times: every problem on R^T R = A^T A (computed in double
    on the device), sampled problems against the oracle."""
    require_gpu()
    ms, ns = inputs.batched_tsqr_sizes()
    seed = inputs.SEEDS["batched_tsqr"]
    As = [inputs.gaussian_device(int(m), int(n), seed * 100003 + i).float() for i, (m, n) in enumerate(zip(ms, ns))]
    As = [a.t().contiguous().t() for a in As]
    grams = [a.double().t() @ a.double() for a in As]
    order = np.argsort(ms)
    sample = sorted(set(order[:: len(order) // 8].tolist() + [int(order[-1]), int(order[0])]))
    host = {i: As[i].cpu().numpy().astype(np.float64) for i in sample}
    banner(f"f32 full batch: {len(As)} problems")
    caqr.tune_batched(dtype=torch.float32)
    B = caqr.tsqr_batched(As)
    torch.cuda.synchronize()
    worst = 0.0
    for a, g in zip(As, grams):
        n = a.shape[1]
        R = torch.triu(a[:n, :n]).double()
        worst = max(worst, float(torch.linalg.norm(R.t() @ R - g) / torch.linalg.norm(g)))
    banner(f"f32 worst Gram residual {worst:.3e}")
    assert worst <= TOL32
    oracle.set_threads(16)
    for i in sample:
        n = int(ns[i])
        R = np.triu(As[i][:n, :n].cpu().numpy()).astype(np.float64)
        assert oracle.rel_fro(R, oracle.qr_r(host[i])) <= TOL32, (i, ms[i], n)
    B.close()
