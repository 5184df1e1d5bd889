"""Pins of the oracle's report layer: single dependency coverage (Sec. 6)
and per-optimizer hotspots (Sec. 7) on hand-worked programs (tests/golden)."""
import json
import os

import pytest

from asm import assemble, samples
from oracle import oracle as O
from paper_2009_04061_amd import synth as S

GOLD = os.path.join(os.path.dirname(__file__), "golden")
NONE = 0xFFFFFFFF


def load(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def recs(spec):
    return samples([(pc, S.STALL_NAMES.index(st), lam, n) for pc, st, lam, n in spec])


def test_single_dependency_coverage_before_and_after_pruning():
    g = load("report_coverage.json")
    prog = assemble(g["program"])
    assert len(prog["op_class"]) == g["expect"]["n_instr"]
    b, a = O.coverage(O.Program(prog))
    assert (b, a) == (g["expect"]["single_before"], g["expect"]["single_after"])


HOT = load("report_hotspots.json")["cases"]


@pytest.mark.parametrize("case", range(len(HOT)),
                         ids=[f"{c['fixture']}:{c['optimizer']}" for c in HOT])
def test_hotspots_hand_worked(case):
    c = HOT[case]
    g = load(c["fixture"])
    prog = assemble(g["program"])
    P = O.Program(prog)
    C, _ = O.count(P.n_instr, recs(g["samples"]))
    bl = P.blame(C)
    got = O.hotspots(P, C, bl, 0, S.OPTIMIZER_NAMES.index(c["optimizer"]), k=5)
    want = [(NONE if r[0] is None else r[0], r[1], r[2], r[3], r[4]) for r in c["expect"]]
    assert [g_[:4] for g_ in got] == [w[:4] for w in want]
    for g_, w in zip(got, want):
        assert g_[4] == pytest.approx(w[4], rel=1e-14)
