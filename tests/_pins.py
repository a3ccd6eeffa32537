"""Pins of the oracle: checks against what the mathematics fixes, not against itself.

Each pin takes the path of an oracle build and returns ``(ok, detail)`` so the
same pins can be run on the real oracle (all must pass) and on builds with a
planted mistake (at least one must fail).  See ``test_oracle_pins.py``.
"""
from __future__ import annotations

import numpy as np

import oracle
from tests import _exact

U = np.finfo(np.float64).eps / 2  # unit roundoff 2^-53


def _res(ok, detail):
    return bool(ok), detail


def pin_bruteforce(lib):
    """R of tiny random inputs vs the Cholesky factor of the exact Gram matrix (60 digits)."""
    rng = np.random.default_rng(11)
    worst = 0.0
    for (m, n) in [(1, 1), (2, 1), (2, 2), (3, 2), (5, 3), (8, 8), (17, 5), (33, 7), (64, 8), (40, 1)]:
        A = rng.standard_normal((m, n))
        Rstar = _exact.cholesky_r(A)
        R = oracle.qr(A, lib).R
        kappa = np.linalg.cond(A) if n > 1 else 1.0
        err = oracle.rel_fro(R, Rstar)
        bound = 10 * n * kappa * U
        worst = max(worst, err / bound)
        if not err <= bound:
            return _res(False, f"m={m} n={n} err={err:.3e} bound={bound:.3e}")
    return _res(True, f"worst err/bound {worst:.3f}")


def pin_closed_forms(lib):
    """n = 1 (R = ||a||, Q = a/||a||), a 2x1 Givens, and the zero matrix."""
    rng = np.random.default_rng(12)
    a = rng.standard_normal((37, 1))
    f = oracle.qr(a, lib)
    nrm = _exact.mp_norm2(a[:, 0])
    if abs(f.R[0, 0] - nrm) > 4 * U * nrm:
        return _res(False, f"n=1 R={f.R[0, 0]!r} vs {nrm!r}")
    if oracle.rel_fro(f.q_thin(), a / nrm) > 8 * U * 37:
        return _res(False, "n=1 Q")
    for (x, y) in [(3.0, 4.0), (-3.0, 4.0), (0.0, -2.0), (1e-300, 1e-300), (1e300, -1e300)]:
        R = oracle.qr(np.array([[x], [y]]), lib).R[0, 0]
        if abs(R - np.hypot(x, y)) > 2 * U * np.hypot(x, y):
            return _res(False, f"givens {x},{y}: {R!r}")
    Z = np.zeros((9, 4))
    fz = oracle.qr(Z, lib)
    if np.any(fz.R != 0) or np.any(fz.beta[:4] != 0):
        return _res(False, "zero matrix R/beta")
    if np.any(fz.q_thin() != np.eye(9, 4)):
        return _res(False, "zero matrix Q")
    return _res(True, "ok")


def pin_upper_triangular(lib):
    """An upper-triangular input with mixed-sign diagonal gives R = D A(0:n, :) bitwise."""
    rng = np.random.default_rng(13)
    n, m = 7, 12
    A = np.zeros((m, n))
    A[:n] = np.triu(rng.standard_normal((n, n)))
    d = np.sign(np.diag(A[:n]))
    R = oracle.qr(A, lib).R
    ok = np.array_equal(R, d[:, None] * A[:n])
    return _res(ok, "bitwise" if ok else f"max diff {np.abs(R - d[:, None] * A[:n]).max():.3e}")


def pin_dyadic(lib):
    """Exact constructions: rows of R0 spread over four distant row blocks, and signed permutations."""
    for (m, n, seed) in [(1024, 8, 1), (1024, 32, 2), (256, 64, 3)]:
        A, R0 = _exact.dyadic_case(m, n, seed)
        R = oracle.qr(A, lib).R
        err = oracle.rel_fro(R, R0)
        if not err <= 50 * n * U:
            return _res(False, f"dyadic m={m} n={n} err={err:.3e}")
    for (m, n, seed) in [(300, 20, 4), (50, 50, 5)]:
        A, R0 = _exact.signed_permutation_case(m, n, seed)
        R = oracle.qr(A, lib).R
        err = oracle.rel_fro(R, R0)
        if not err <= 50 * n * U:
            return _res(False, f"signed permutation m={m} n={n} err={err:.3e}")
    return _res(True, "ok")


def pin_lapack(lib):
    """LAPACK (numpy.linalg.qr) R, sign-normalized, within 1e-13 normwise."""
    rng = np.random.default_rng(14)
    for (m, n) in [(500, 40), (129, 64), (64, 64)]:
        A = rng.standard_normal((m, n))
        Rl = np.linalg.qr(A, mode="r")
        Rl = np.sign(np.diag(Rl))[:, None] * Rl
        err = oracle.rel_fro(oracle.qr(A, lib).R, Rl)
        if not err <= 1e-13:
            return _res(False, f"m={m} n={n} err={err:.3e}")
    return _res(True, "ok")


def pin_invariants(lib):
    """||A - QR||/||A|| and ||I - Q^T Q|| at O(eps); R(2^k A) = 2^k R(A) bitwise."""
    rng = np.random.default_rng(15)
    A = rng.standard_normal((700, 48))
    f = oracle.qr(A, lib)
    Q = f.q_thin()
    e1, e2 = oracle.factorization_error(A, Q, f.R), oracle.orthogonality_error(Q)
    if not (e1 <= 1e-14 and e2 <= 1e-13):
        return _res(False, f"||A-QR||={e1:.3e} ||I-QtQ||={e2:.3e}")
    for k in (-1000, -600, -3, 5, 700, 1000):
        if not np.array_equal(oracle.qr(np.ldexp(A, k), lib).R, np.ldexp(f.R, k)):
            return _res(False, f"scaling by 2^{k} not exact")
    # subnormal input: the norm's power-of-two scaling must stay finite
    As = np.ldexp(A[:50, :6], -1060)
    Rs = oracle.qr(As, lib).R
    if not np.all(np.isfinite(Rs)):
        return _res(False, "subnormal input gives a non-finite R")
    if oracle.rel_fro(np.ldexp(np.abs(np.diag(Rs)), 1060), np.abs(np.diag(oracle.qr(np.ldexp(As, 1060), lib).R))) > 1e-3:
        return _res(False, "subnormal input: wrong R diagonal")
    # apply_q(apply_qt(C)) = C
    C = rng.standard_normal((700, 5))
    back = f.apply_q(f.apply_qt(C))
    if oracle.rel_fro(back, C) > 1e-14:
        return _res(False, "apply_q o apply_qt != I")
    return _res(True, f"{e1:.2e} {e2:.2e}")


def pin_ls(lib):
    """Least squares vs the exact rational solution, and a consistent system with a known x."""
    rng = np.random.default_rng(16)
    for (m, n) in [(9, 3), (20, 6), (31, 8)]:
        A = rng.standard_normal((m, n))
        b = rng.standard_normal(m)
        xs = _exact.exact_ls(A, b)
        x, st = oracle.ls(A, b, lib)
        if st != 0:
            return _res(False, f"status {st}")
        kappa = np.linalg.cond(A)
        r = b - A @ xs
        bound = 50 * n * (kappa * U + kappa ** 2 * U * np.linalg.norm(r) / (np.linalg.norm(A, 2) * np.linalg.norm(xs)))
        err = np.linalg.norm(x[:, 0] - xs) / np.linalg.norm(xs)
        if not err <= bound:
            return _res(False, f"m={m} n={n} err={err:.3e} bound={bound:.3e}")
    A = rng.standard_normal((400, 30))
    xt = rng.standard_normal(30)
    x, st = oracle.ls(A, A @ xt, lib)
    if oracle.rel_fro(x[:, 0], xt) > 1e-13:
        return _res(False, "consistent system")
    eta = oracle.ls_eta(A, x, A @ xt)
    if eta > 1e-15:
        return _res(False, f"eta {eta:.3e}")
    Z = rng.standard_normal((10, 3))
    Z[:, 1] = 0.0
    _, st = oracle.ls(Z, rng.standard_normal(10), lib)
    if st != 2:
        return _res(False, f"singular status {st}")
    return _res(True, "ok")


def pin_ls_eta(lib, eta=None):
    """The least-squares backward-error measure against its definition evaluated
    exactly: residual and A^T r in rationals, 2-norms and ||A||_2 (largest
    singular value, from the exact Gram matrix) at 60 digits.  Inconsistent
    systems (b not in the range of A) at points x away from the solution, where
    A^T r is far from zero, and near it (x = x* + a small perturbation), where
    it is small but not zero; ||A||_2 computed by the function and passed in."""
    eta = oracle.ls_eta if eta is None else eta
    rng = np.random.default_rng(17)
    for (m, n, scale) in [(7, 3, 1.0), (12, 5, 1e-3), (20, 4, 1.0), (9, 1, 1.0), (15, 6, 1e-8)]:
        A = rng.standard_normal((m, n))
        b = rng.standard_normal(m)  # almost surely not in the range of A
        xs = _exact.exact_ls(A, b)
        for x in (xs + scale * rng.standard_normal(n), rng.standard_normal(n)):
            ref = _exact.exact_eta(A, x, b)
            for norm_a in (None, float(np.linalg.norm(A, 2))):
                got = eta(A, x, b, norm_a=norm_a)
                # FP64 evaluation: the residual's rounding (about u ||b||) relative
                # to ||A^T r|| bounds the error of the numerator
                tol = 1e-12 * ref + 64 * U * np.linalg.norm(A, 2) * np.linalg.norm(b) / (
                    np.linalg.norm(A, 2) * (np.linalg.norm(A, 2) * np.linalg.norm(x) + np.linalg.norm(b)))
                if not abs(got - ref) <= tol:
                    return _res(False, f"m={m} n={n} eta={got!r} exact={ref!r}")
    return _res(True, "ok")


ALL_PINS = [pin_bruteforce, pin_closed_forms, pin_upper_triangular, pin_dyadic, pin_lapack, pin_invariants, pin_ls,
            pin_ls_eta]
