"""Exact and extended-precision references used to pin the oracle.

Doubles are exact rationals, so A^T A and A^T b are computed exactly with
``fractions.Fraction``; the Cholesky factor of A^T A (which is the R of A with a
positive diagonal) is then taken in mpmath at 60 significant digits.  Nothing
here shares code with the oracle or with the GPU library.
"""
from __future__ import annotations

from fractions import Fraction

import mpmath
import numpy as np


def exact_gram(A: np.ndarray):
    m, n = A.shape
    cols = [[Fraction(float(A[i, j])) for i in range(m)] for j in range(n)]
    G = [[None] * n for _ in range(n)]
    for a in range(n):
        for b in range(a, n):
            s = sum((x * y for x, y in zip(cols[a], cols[b])), Fraction(0))
            G[a][b] = G[b][a] = s
    return G


def cholesky_r(A: np.ndarray, dps: int = 60) -> np.ndarray:
    """R (upper, positive diagonal) with R^T R = A^T A, to `dps` digits, rounded to double."""
    G = exact_gram(A)
    n = len(G)
    with mpmath.workdps(dps):
        Gm = [[mpmath.mpf(g.numerator) / g.denominator for g in row] for row in G]
        R = [[mpmath.mpf(0)] * n for _ in range(n)]
        for j in range(n):
            s = Gm[j][j] - sum((R[i][j] ** 2 for i in range(j)), mpmath.mpf(0))
            R[j][j] = mpmath.sqrt(s)
            for k in range(j + 1, n):
                t = Gm[j][k] - sum((R[i][j] * R[i][k] for i in range(j)), mpmath.mpf(0))
                R[j][k] = t / R[j][j]
        return np.array([[float(R[i][j]) for j in range(n)] for i in range(n)])


def exact_ls(A: np.ndarray, b: np.ndarray) -> np.ndarray:
    """x* = (A^T A)^{-1} A^T b, solved exactly in rationals (Gauss-Jordan)."""
    m, n = A.shape
    G = exact_gram(A)
    rhs = [sum((Fraction(float(A[i, j])) * Fraction(float(b[i])) for i in range(m)), Fraction(0)) for j in range(n)]
    M = [row[:] + [rhs[j]] for j, row in enumerate(G)]
    for c in range(n):
        p = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[p] = M[p], M[c]
        piv = M[c][c]
        M[c] = [v / piv for v in M[c]]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c]
                M[r] = [vr - f * vc for vr, vc in zip(M[r], M[c])]
    return np.array([float(M[j][n]) for j in range(n)])


def mp_norm2(v) -> float:
    with mpmath.workdps(60):
        s = sum((Fraction(float(x)) ** 2 for x in v), Fraction(0))
        return float(mpmath.sqrt(mpmath.mpf(s.numerator) / s.denominator))


def dyadic_case(m: int, n: int, seed: int = 0):
    """A = (prod_k H_k) [R0; 0] built exactly in binary.

    R0 is a small-integer upper triangle with a positive diagonal.  For every
    row k < n, H_k = I - (1/2) u_k u_k^T with u_k = +-1 on the four rows
    k, L+k, 2L+k, 3L+k (L = m // 4), so u_k^T u_k = 4 and H_k is orthogonal and
    exact in floating point; the supports are disjoint, so the product is exact
    too.  Each row of R0 is thereby spread over four distant row blocks (and so
    over different leaves of any row-block tree).  The unique R of A is R0.
    """
    L = m // 4
    if n > L:
        raise ValueError("need n <= m // 4")
    rng = np.random.default_rng(seed)
    R0 = np.triu(rng.integers(-4, 5, size=(n, n))).astype(np.float64)
    R0[np.arange(n), np.arange(n)] = rng.integers(1, 6, size=n)
    A = np.zeros((m, n))
    A[:n] = R0
    for k in range(n):
        rows = [k, L + k, 2 * L + k, 3 * L + k]
        u = rng.choice([-1.0, 1.0], size=4)
        blk = A[rows, :]
        A[rows, :] = blk - 0.5 * np.outer(u, u @ blk)  # exact half-integers
    return np.asfortranarray(A), R0


def signed_permutation_case(m: int, n: int, seed: int = 0):
    """A = P S [R0; 0] with P a row permutation and S = diag(+-1): R(A) = R0."""
    rng = np.random.default_rng(seed)
    R0 = np.triu(rng.standard_normal((n, n)))
    R0[np.arange(n), np.arange(n)] = np.abs(R0[np.arange(n), np.arange(n)]) + 0.5
    X = np.zeros((m, n))
    X[:n] = R0
    X *= rng.choice([-1.0, 1.0], size=(m, 1))
    return np.asfortranarray(X[rng.permutation(m)]), R0


def exact_eta(A: np.ndarray, x: np.ndarray, b: np.ndarray, dps: int = 60) -> float:
    """eta(x) = ||A^T (b - A x)||_2 / (||A||_2 (||A||_2 ||x||_2 + ||b||_2)) with the
    residual and A^T r exact in rationals, and the 2-norms (||A||_2 as the square
    root of the largest eigenvalue of the exact A^T A) at `dps` digits."""
    m, n = A.shape
    Af = [[Fraction(float(A[i, j])) for j in range(n)] for i in range(m)]
    xf = [Fraction(float(v)) for v in np.ravel(x)]
    bf = [Fraction(float(v)) for v in np.ravel(b)]
    r = [bf[i] - sum((Af[i][j] * xf[j] for j in range(n)), Fraction(0)) for i in range(m)]
    g = [sum((Af[i][j] * r[i] for i in range(m)), Fraction(0)) for j in range(n)]
    G = exact_gram(A)
    with mpmath.workdps(dps):
        mp = lambda q: mpmath.mpf(q.numerator) / q.denominator
        nrm = lambda v: mpmath.sqrt(mp(sum((q * q for q in v), Fraction(0))))
        ev = mpmath.eigsy(mpmath.matrix([[mp(q) for q in row] for row in G]), eigvals_only=True)
        na = mpmath.sqrt(max(ev[i] for i in range(n)))
        return float(nrm(g) / (na * (na * nrm(xf) + nrm(bf))))
