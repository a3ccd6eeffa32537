"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module only draws random numbers and lays them out; it holds none of the
factorization's arithmetic.  Every matrix is column-major (Fortran order), and
``standard_normal`` fills it in column-major order: element (i, j) is draw
number ``j*m + i`` of a ``numpy.random.default_rng(seed)`` (PCG64) stream.
"""
from __future__ import annotations

import numpy as np

# One seed per workload; sub-streams come from SeedSequence(seed).spawn.
SEEDS = {
    "tsqr_4096x32": 1,
    "caqr_8192sq": 2,
    "tsqr_1Mx64": 3,
    "batched_tsqr": 4,
    "mixed_ls": 5,
    "served_ls": 6,
}


def gaussian(m: int, n: int, seed: int, dtype=np.float64) -> np.ndarray:
    """m-by-n iid N(0,1), column-major draw order, Fortran layout."""
    rng = np.random.default_rng(seed)
    a = rng.standard_normal(m * n).reshape(n, m).T  # (i, j) = draw j*m + i
    a = np.asfortranarray(a)
    if dtype != np.float64:
        a = np.asfortranarray(a.astype(dtype))  # round-to-nearest of the same draws
    return a


def substreams(seed: int, k: int) -> list[np.random.Generator]:
    return [np.random.default_rng(s) for s in np.random.SeedSequence(seed).spawn(k)]


def log_uniform_int(rng: np.random.Generator, lo: int, hi: int, size: int) -> np.ndarray:
    """Integers round(exp(U[ln lo, ln hi]))."""
    return np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi), size))).astype(np.int64)


def batched_tsqr_sizes(count: int = 2000, seed: int = SEEDS["batched_tsqr"]):
    """Sizes of the uneven batch: m log-uniform in [256, 65536], n uniform on {8,16,32,64}."""
    rng = np.random.default_rng(seed)
    m = log_uniform_int(rng, 256, 65536, count)
    n = rng.choice(np.array([8, 16, 32, 64]), size=count)
    return m, n


def geometric_singular_values(n: int, kappa: float) -> np.ndarray:
    """s_i = kappa^(-(i-1)/(n-1)), i = 1..n, so s_1 = 1 and s_n = 1/kappa."""
    if n == 1:
        return np.ones(1)
    return kappa ** (-np.arange(n) / (n - 1.0))


def gaussian_device(m: int, n: int, seed: int, device="cuda"):
    """N(0,1) m-by-n matrix drawn on the GPU (torch's seeded generator), column
    major: for inputs too large to draw on the host (the full uneven batch)."""
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(seed)
    return torch.randn((n, m), generator=g, dtype=torch.float64, device=device).t()


def served_ls_requests(count: int = 512, seed: int = SEEDS["served_ls"]):
    """Request mix of the served least-squares stream: m log-uniform in
    [1024, 262144], n log-uniform in [16, 512], condition number kappa
    log-uniform in [1e2, 1e6]."""
    rng = np.random.default_rng(seed)
    m = log_uniform_int(rng, 1024, 262144, count)
    n = np.minimum(log_uniform_int(rng, 16, 512, count), m)
    kappa = np.exp(rng.uniform(np.log(1e2), np.log(1e6), count))
    return m, n, kappa


def poisson_arrivals(rate: float, duration: float, seed: int) -> np.ndarray:
    """Arrival times (seconds) of a Poisson process of the given rate on [0, duration)."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, int(rate * duration * 1.5) + 16))
    return t[t < duration]


def conditioned_device(m: int, n: int, kappa: float, seed: int, device="cuda"):
    """A = G diag(s) V^T on the device, column-major: G an m-by-n N(0,1) draw
    (torch's seeded generator), s geometric from 1 to 1/kappa, V the orthogonal
    factor of an n-by-n N(0,1) draw (numpy's QR); the singular values of A
    spread over about kappa times those of G."""
    import torch

    G = gaussian_device(m, n, seed, device)
    rng = np.random.default_rng(seed)
    V = np.linalg.qr(rng.standard_normal((n, n)))[0]
    s = geometric_singular_values(n, kappa)
    W = torch.as_tensor(np.ascontiguousarray((V * s).T), device=device)  # diag(s) V^T, row-major n x n
    A = torch.empty((n, m), dtype=torch.float64, device=device).t()
    torch.matmul(G, W, out=A)
    return A


def conditioned_host(m: int, n: int, kappa: float, seed: int) -> np.ndarray:
    """A = U diag(s) V^T on the host, column-major: U the orthonormal factor of
    an m-by-n N(0,1) draw and V of an n-by-n one (host LAPACK QR, input
    construction only), s geometric from 1 to 1/kappa, so ||A||_2 = 1 and
    kappa(A) = kappa (the mixed-precision least-squares configuration)."""
    rngs = substreams(seed, 2)
    U = np.linalg.qr(rngs[0].standard_normal((m, n)))[0]
    V = np.linalg.qr(rngs[1].standard_normal((n, n)))[0]
    s = geometric_singular_values(n, kappa)
    return np.asfortranarray((U * s) @ V.T)
