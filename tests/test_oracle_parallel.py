"""Pins of the oracle's parallel estimators (Sec. 5.2, Eqs. (6)-(10)) against
hand-worked cases whose values are exact fractions (tests/golden)."""
import json
import os

import pytest

from asm import assemble, samples
from oracle import oracle as O
from paper_2009_04061_amd import synth as S

GOLD = os.path.join(os.path.dirname(__file__), "golden", "parallel_estimators.json")


def load():
    with open(GOLD) as f:
        return json.load(f)


def value(v):
    return v[0] / v[1] if isinstance(v, list) else float(v)


def oracle_case(g, c):
    prog = assemble(g["program"])
    rec = samples([(pc, S.STALL_NAMES.index(st), lam, n) for pc, st, lam, n in c["samples"]])
    P = O.Program(prog)
    C, _ = O.count(P.n_instr, rec)
    return O.parallel(P, C, 0, c["launch"], g["device"])


CASES = load()["cases"]


@pytest.mark.parametrize("case", range(len(CASES)), ids=[c["name"] for c in CASES])
def test_parallel_estimators_hand_worked(case):
    g = load()
    c = g["cases"][case]
    got = oracle_case(g, c)
    for o, want in enumerate(c["expect"]):
        for key, v in want.items():
            assert got[o][key] == pytest.approx(value(v), rel=1e-14, abs=1e-15), (o, key)
