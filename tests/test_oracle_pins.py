"""The oracle pinned to what the paper and the mathematics fix (CPU only).

Every pin in ``_pins`` must pass on the oracle, and every planted mistake
(compiled in with -DORACLE_MUTANT=k) must be caught by at least one pin.
"""
import os

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
