"""The oracle pinned to what the paper and the mathematics fix (CPU only).

Every pin in ``_pins`` must pass on the oracle, and every planted mistake
(compiled in with -DORACLE_MUTANT=k) must be caught by at least one pin.
"""
import os

import numpy as np
import pytest

import oracle
from tests import _pins


@pytest.mark.parametrize("pin", _pins.ALL_PINS, ids=lambda p: p.__name__)
def test_pin(pin, oracle_mod):
    ok, detail = pin(oracle.LIB)
    assert ok, detail


MUTANTS = {
    1: "drop a term of sigma",
    2: "wrong sign in v(1)",
    3: "drop the implicit unit of v in v^T c",
    4: "skip a trailing column",
    5: "Q^T applied in the wrong order",
    6: "Q applied in the wrong order",
    7: "transposed R in back substitution",
}


@pytest.mark.parametrize("k", sorted(MUTANTS), ids=lambda k: MUTANTS[k])
def test_planted_mistake_is_caught(k, tmp_path):
    path = oracle.build(str(tmp_path / f"liboracle_m{k}.so"), mutant=k)
    failed = []
    for pin in _pins.ALL_PINS:
        try:
            ok, _ = pin(path)
        except Exception:  # a crash or a raised error also counts as caught
            ok = False
        if not ok:
            failed.append(pin.__name__)
    assert failed, f"mutant {k} ({MUTANTS[k]}) passed every pin"


def _eta_parts(A, x, b, norm_a=None):
    A = np.asarray(A, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64).reshape(A.shape[1], -1)
    b = np.asarray(b, dtype=np.float64).reshape(A.shape[0], -1)
    na = float(np.linalg.norm(A, 2)) if norm_a is None else norm_a
    return A, x, b, na, b - A @ x


def _eta_no_at(A, x, b, norm_a=None):  # A^T dropped from the numerator
    A, x, b, na, r = _eta_parts(A, x, b, norm_a)
    return float(np.max(np.linalg.norm(r, axis=0) / (na * (na * np.linalg.norm(x, axis=0) + np.linalg.norm(b, axis=0)))))


def _eta_one_norm_a(A, x, b, norm_a=None):  # ||A|| once instead of twice in front of ||x||
    A, x, b, na, r = _eta_parts(A, x, b, norm_a)
    return float(np.max(np.linalg.norm(A.T @ r, axis=0) / (na * (np.linalg.norm(x, axis=0) + np.linalg.norm(b, axis=0)))))


def _eta_no_b(A, x, b, norm_a=None):  # ||b|| dropped from the denominator
    A, x, b, na, r = _eta_parts(A, x, b, norm_a)
    return float(np.max(np.linalg.norm(A.T @ r, axis=0) / (na * na * np.linalg.norm(x, axis=0))))


def _eta_frobenius(A, x, b, norm_a=None):  # Frobenius norm of A in place of the 2-norm
    A, x, b, _, r = _eta_parts(A, x, b, None)
    na = float(np.linalg.norm(A)) if norm_a is None else norm_a
    return float(np.max(np.linalg.norm(A.T @ r, axis=0) / (na * (na * np.linalg.norm(x, axis=0) + np.linalg.norm(b, axis=0)))))


ETA_MUTANTS = {"drop A^T": _eta_no_at, "one factor ||A||": _eta_one_norm_a, "drop ||b||": _eta_no_b,
               "Frobenius norm": _eta_frobenius}


@pytest.mark.parametrize("name", sorted(ETA_MUTANTS))
def test_planted_eta_mistake_is_caught(name, oracle_mod):
    """Each planted mistake in the backward-error measure fails its pin."""
    ok, _ = _pins.pin_ls_eta(oracle.LIB, eta=ETA_MUTANTS[name])
    assert not ok, f"eta mutant '{name}' passed the pin"
