"""Pin strength: each planted mistake in the oracle fails at least one pin.

The oracle is rebuilt with -DORACLE_MUTANT=k (a conjugated operand, a dropped
term, a transposed operand, a flipped twiddle sign, padding one short of the
minimal length, a wrong normalisation, the wrong root of unity, a centered
operand read one place off, a centre rounded up instead of down, a Hermitian
mirror without the conjugate) and the pins
of tests/test_oracle.py are run against each build; every build must fail at
least one of them.  The default build is checked to pass them all.
"""
import inspect
import os

import pytest

import oracle
import test_oracle as pins

MUTANTS = {1: "conjugated operand", 2: "dropped term", 3: "transposed operand",
           4: "twiddle sign", 5: "padding too short", 6: "normalisation", 7: "root of unity",
           8: "centered operand off by one", 9: "centre rounded up", 10: "Hermitian mirror without conjugate"}


def _pin_calls():
    calls = []
    for name, fn in inspect.getmembers(pins, inspect.isfunction):
        if not name.startswith("test_"):
            continue
        marks = getattr(fn, "pytestmark", [])
        params = [m for m in marks if m.name == "parametrize"]
        if not params:
            calls.append((name, fn, {}))
            continue
        m = params[0]
        argnames = [a.strip() for a in m.args[0].split(",")]
        for vals in m.args[1]:
            vals = vals if len(argnames) > 1 else (vals,)
            calls.append((name, fn, dict(zip(argnames, vals))))
    return calls


def _failures():
    bad = []
    for name, fn, kw in _pin_calls():
        try:
            fn(**kw)
        except Exception:
            bad.append((name, kw))
    return bad


@pytest.mark.parametrize("k", sorted(MUTANTS))
def test_mutant_is_caught(k, tmp_path):
    path = oracle.build(out=str(tmp_path / ("liboracle_m%d.so" % k)), defines=["ORACLE_MUTANT=%d" % k])
    try:
        oracle.use_library(path)
        bad = _failures()
    finally:
        oracle.use_library(None)
    assert bad, "planted mistake %d (%s) passed every pin" % (k, MUTANTS[k])


def test_default_build_passes_all_pins():
    assert _failures() == []
