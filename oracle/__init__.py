"""Householder QR oracle: TEST INFRASTRUCTURE ONLY.

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never does, and the
oracle shares no code with it.

The arithmetic lives in ``oracle_qr.c`` (plain C, FP64): the textbook
column-by-column Householder QR that defines what the multilevel method of the
paper (Section 3.1, Algorithm 1) computes.  This module only loads that code and
marshals numpy arrays, plus the error metrics the tests use.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "oracle_qr.c")
LIB = os.path.join(_HERE, "liboracle.so")

_c_i64 = ctypes.c_int64
_c_dp = ctypes.POINTER(ctypes.c_double)


def build(out: str = LIB, mutant: int = 0) -> str:
    """Compile the oracle (gcc -O2, no fast-math, OpenMP).

    ``mutant`` != 0 plants one of the deliberate mistakes used by the
    pin-strength tests; such builds go to a separate file and are never the
    oracle itself.
    """
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", f"-DORACLE_MUTANT={int(mutant)}",
           SRC, "-o", out + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


_libs: dict[str, ctypes.CDLL] = {}


def load(path: str = LIB) -> ctypes.CDLL:
    if path in _libs:
        return _libs[path]
    if not os.path.exists(path):
        if path != LIB:
            raise FileNotFoundError(path)
        build(path)
    lib = ctypes.CDLL(path)
    for name in ("oracle_qr",):
        getattr(lib, name).argtypes = [_c_i64, _c_i64, _c_dp, _c_i64, _c_dp]
        getattr(lib, name).restype = ctypes.c_int
    for name in ("oracle_apply_qt", "oracle_apply_q"):
        getattr(lib, name).argtypes = [_c_i64, _c_i64, _c_dp, _c_i64, _c_dp, _c_i64, _c_dp, _c_i64]
        getattr(lib, name).restype = ctypes.c_int
    lib.oracle_form_q.argtypes = [_c_i64, _c_i64, _c_dp, _c_i64, _c_dp, _c_dp, _c_i64]
    lib.oracle_form_q.restype = ctypes.c_int
    lib.oracle_trsm_upper.argtypes = [_c_i64, _c_dp, _c_i64, _c_i64, _c_dp, _c_i64]
    lib.oracle_trsm_upper.restype = ctypes.c_int
    lib.oracle_ls.argtypes = [_c_i64, _c_i64, _c_i64, _c_dp, _c_i64, _c_dp, _c_i64, _c_dp]
    lib.oracle_ls.restype = ctypes.c_int
    lib.oracle_num_threads.restype = ctypes.c_int
    lib.oracle_set_threads.argtypes = [ctypes.c_int]
    _libs[path] = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_c_dp)


def _fortran(a) -> np.ndarray:
    return np.array(a, dtype=np.float64, order="F", copy=True)


class Factorization:
    """Result of :func:`qr`: ``F`` holds R (upper) and the reflectors (below)."""

    def __init__(self, F: np.ndarray, beta: np.ndarray, lib: ctypes.CDLL):
        self.F, self.beta, self._lib = F, beta, lib
        self.m, self.n = F.shape

    @property
    def R(self) -> np.ndarray:
        return np.triu(self.F[: self.n, : self.n])

    def q_thin(self) -> np.ndarray:
        Q = np.zeros((self.m, self.n), order="F")
        rc = self._lib.oracle_form_q(self.m, self.n, _ptr(self.F), self.m, _ptr(self.beta), _ptr(Q), max(1, self.m))
        assert rc == 0
        return Q

    def apply_qt(self, C) -> np.ndarray:
        C = _fortran(C).reshape(self.m, -1, order="F")
        rc = self._lib.oracle_apply_qt(self.m, self.n, _ptr(self.F), self.m, _ptr(self.beta), C.shape[1], _ptr(C),
                                       max(1, self.m))
        assert rc == 0
        return C

    def apply_q(self, C) -> np.ndarray:
        C = _fortran(C).reshape(self.m, -1, order="F")
        rc = self._lib.oracle_apply_q(self.m, self.n, _ptr(self.F), self.m, _ptr(self.beta), C.shape[1], _ptr(C),
                                      max(1, self.m))
        assert rc == 0
        return C


def qr(A, lib_path: str = LIB) -> Factorization:
    """Householder QR of an m-by-n (m >= n) matrix; R has a non-negative diagonal."""
    lib = load(lib_path)
    F = _fortran(A)
    if F.ndim != 2:
        raise ValueError("A must be 2-D")
    m, n = F.shape
    beta = np.zeros(max(n, 1))
    rc = lib.oracle_qr(m, n, _ptr(F), max(1, m), _ptr(beta))
    if rc != 0:
        raise ValueError(f"oracle_qr rejected m={m}, n={n}")
    return Factorization(F, beta, lib)


def qr_r(A, lib_path: str = LIB) -> np.ndarray:
    return qr(A, lib_path).R


def ls(A, B, lib_path: str = LIB):
    """Least squares via QR; returns (X (n-by-nrhs), status) with status 1+j for a zero R_jj."""
    lib = load(lib_path)
    F = _fortran(A)
    m, n = F.shape
    Bf = _fortran(B).reshape(m, -1, order="F")
    beta = np.zeros(max(n, 1))
    rc = lib.oracle_ls(m, n, Bf.shape[1], _ptr(F), max(1, m), _ptr(Bf), max(1, m), _ptr(beta))
    if rc < 0:
        raise ValueError("oracle_ls rejected its arguments")
    return Bf[:n].copy(), rc


def set_threads(t: int) -> None:
    load().oracle_set_threads(int(t))


def num_threads() -> int:
    return int(load().oracle_num_threads())


# ----------------------------------------------------------------------------------------------
# metrics (definitions, used by every test and by the benchmark's parity checks)
# ----------------------------------------------------------------------------------------------
def rel_fro(X, Xref) -> float:
    """||X - Xref||_F / ||Xref||_F (absolute when Xref == 0)."""
    X = np.asarray(X, dtype=np.float64)
    Xref = np.asarray(Xref, dtype=np.float64)
    den = np.linalg.norm(Xref)
    num = np.linalg.norm(X - Xref)
    return float(num / den) if den > 0 else float(num)


def factorization_error(A, Q, R) -> float:
    """||A - Q R||_F / ||A||_F."""
    return rel_fro(np.asarray(Q) @ np.asarray(R), A)


def orthogonality_error(Q) -> float:
    """||I - Q^T Q||_F."""
    Q = np.asarray(Q, dtype=np.float64)
    return float(np.linalg.norm(np.eye(Q.shape[1]) - Q.T @ Q))


def ls_eta(A, x, b, norm_a: float | None = None) -> float:
    """Normwise backward-error proxy for least squares:
    ||A^T (b - A x)||_2 / (||A||_2 (||A||_2 ||x||_2 + ||b||_2)), in FP64."""
    A = np.asarray(A, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64).reshape(A.shape[1], -1)
    b = np.asarray(b, dtype=np.float64).reshape(A.shape[0], -1)
    if norm_a is None:
        norm_a = float(np.linalg.norm(A, 2))
    r = b - A @ x
    num = np.linalg.norm(A.T @ r, axis=0)
    den = norm_a * (norm_a * np.linalg.norm(x, axis=0) + np.linalg.norm(b, axis=0))
    return float(np.max(num / den))
