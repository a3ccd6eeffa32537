"""Batched TSQR over uneven problems (one launch per leaf-height / width group):
every problem bitwise equal to a single tsqr_factor call with the same plan, and
within 1e-11 of the oracle; the full 2000-problem batch on sampled problems and
on the Gram identity R^T R = A^T A for every problem."""
import numpy as np
import pytest
import torch

import oracle
from paper_1303_5837_amd import caqr, inputs
from tests._gpu import banner, require_gpu

pytestmark = pytest.mark.gpu

TOL_R = 1e-11

# (m, n): single-leaf, ragged, m == n, widths on and off 16-column slots
SIZES = [(1, 1), (7, 5), (64, 64), (100, 8), (255, 16), (256, 17), (257, 32), (300, 1), (511, 33),
         (700, 64), (1000, 40), (1024, 64), (1500, 8), (2049, 16), (3000, 32), (4096, 64), (5000, 3),
         (333, 0), (6000, 64), (129, 64)]


def make(sizes, seed):
    hosts, devs = [], []
    for i, (m, n) in enumerate(sizes):
        A = inputs.gaussian(m, n, seed + i) if n else np.zeros((m, 0))
        hosts.append(A)
        devs.append(caqr.fortran(A) if n else torch.empty((0, m), dtype=torch.float64, device="cuda").t())
    return hosts, devs


def single(A, plan):
    d = caqr.fortran(A)
    F = caqr.tsqr(d, leaf_rows=plan[0], leaves_per_wg=plan[1], arity=plan[2])
    torch.cuda.synchronize()
    return d.cpu().numpy(), F.signs()


def check_batch(sizes, seed, **plan):
    hosts, devs = make(sizes, seed)
    B = caqr.tsqr_batched(devs, **plan)
    torch.cuda.synchronize()
    for i, (m, n) in enumerate(sizes):
        if n == 0:
            continue
        banner(f"batched problem {i}: m={m} n={n} plan={B.plan(i)}")
        got = devs[i].cpu().numpy()
        R = np.triu(got[:n, :n])
        assert np.all(np.diag(R) >= 0)
        assert oracle.rel_fro(R, oracle.qr_r(hosts[i])) <= TOL_R
        ref, d = single(hosts[i], B.plan(i))
        assert np.array_equal(got, ref), (m, n)        # R, Y and V bitwise
        assert np.array_equal(B.signs(i), d)
    B.close()


def test_fixed_plan_matches_single_and_oracle():
    require_gpu()
    oracle.set_threads(16)
    check_batch(SIZES, 300, leaf_rows=256, leaves_per_wg=4)


@pytest.mark.parametrize("leaf_rows,lpw,arity", [(64, 1, 4), (128, 2, 2), (64, 4, 4), (256, 1, 2), (128, 4, 2)])
def test_other_plans(leaf_rows, lpw, arity):
    require_gpu()
    check_batch(SIZES[:12], 400 + leaf_rows + lpw, leaf_rows=leaf_rows, leaves_per_wg=lpw, arity=arity)


def test_default_plans():
    require_gpu()
    check_batch(SIZES, 500)


def test_tuner_plans_are_used():
    require_gpu()
    caqr.tune_batched()
    sizes = [(300, 8), (5000, 16), (40000, 64), (70000, 32), (100, 64)]
    for m, n in sizes:
        hr, lpw, ar = caqr.batch_plan_for(m, n)
        assert hr in (64, 128, 256) and (ar, lpw) in ((2, 1), (2, 2), (2, 4), (4, 1), (4, 4))
    hosts, devs = make(sizes, 600)
    B = caqr.tsqr_batched(devs)
    torch.cuda.synchronize()
    for i, (m, n) in enumerate(sizes):
        assert B.plan(i) == caqr.batch_plan_for(m, n)
        ref, _ = single(hosts[i], B.plan(i))
        assert np.array_equal(devs[i].cpu().numpy(), ref)
    B.close()


def test_full_uneven_batch_sampled():
    """The uneven batch at full size (2000 problems, m log-uniform in [256, 65536],
    n in {8, 16, 32, 64}, seed 4), in the plan the benchmark times: sampled
    problems against the oracle, every problem on R^T R = A^T A."""
    require_gpu()
    ms, ns = inputs.batched_tsqr_sizes()
    seed = inputs.SEEDS["batched_tsqr"]
    As = [inputs.gaussian_device(int(m), int(n), seed * 100003 + i) for i, (m, n) in enumerate(zip(ms, ns))]
    grams = [a.t() @ a for a in As]
    order = np.argsort(ms)
    sample = sorted(set(order[:: len(order) // 10].tolist() + [int(order[-1]), int(order[0])]))
    host = {i: As[i].cpu().numpy() for i in sample}
    banner(f"full batch: {len(As)} problems, {sum(int(m) * int(n) for m, n in zip(ms, ns)) * 8 / 2**30:.2f} GiB")
    caqr.tune_batched()
    B = caqr.tsqr_batched(As)
    torch.cuda.synchronize()
    worst = 0.0
    for i, (a, g) in enumerate(zip(As, grams)):
        n = a.shape[1]
        R = torch.triu(a[:n, :n])
        worst = max(worst, float(torch.linalg.norm(R.t() @ R - g) / torch.linalg.norm(g)))
    banner(f"worst Gram residual {worst:.3e}")
    assert worst <= 1e-13
    oracle.set_threads(16)
    for i in sample:
        n = int(ns[i])
        R = np.triu(As[i][:n, :n].cpu().numpy())
        assert oracle.rel_fro(R, oracle.qr_r(host[i])) <= TOL_R, (i, ms[i], n)
    B.close()
