"""Pins of the oracle against the paper's worked examples (tests/golden)."""
import json
import os

import numpy as np
import pytest

from asm import assemble, samples, use_index
from oracle import oracle as O
from paper_2009_04061_amd import synth as S

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def load(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def loc(prog, name):
    if name[0] == "R":
        return int(name[1:])
    if name[0] == "P":
        return prog["n_regs"] + int(name[1:])
    return prog["n_regs"] + prog["n_preds"] + int(name[1:])


def recs(spec):
    return samples([(pc, S.STALL_NAMES.index(st), lam, n) for pc, st, lam, n in spec])


def test_fig1_sampling_ratios():
    g = load("fig1_sampling.json")
    prog = assemble(g["program"])
    res = O.run_all(prog, recs(g["samples"]))
    C = res["C"]
    e = g["expect"]
    T = res["estimate"]["kernel_T"][0]
    L = res["estimate"]["kernel_L"][0]
    assert T == e["T"] and L == e["latency"] and T - L == e["active"]
    assert res["estimate"]["active"][0] == e["active"]
    issued = C[:, S.ST_SELECTED, :].sum()
    assert T - issued == e["stall_samples"]
    assert L / T == e["stall_ratio"] and (T - L) / T == e["active_ratio"]


def test_fig3_barrier_dependency():
    g = load("fig3_barrier.json")
    prog = assemble(g["program"])
    P = O.Program(prog)
    u = use_index(prog, g["use"]["instr"], loc(prog, g["use"]["loc"]))
    assert list(P.sources(u)) == g["expect"]["sources"]
    res = O.run_all(prog, recs(g["samples"]))
    bl = res["blame"]
    for i, (a, l) in g["expect"]["blamed_mem_dep"].items():
        assert bl["blamed"][int(i), S.ST_MEM_DEP].tolist() == [a, l]
    assert bl["self"][g["use"]["instr"], S.ST_MEM_DEP].tolist() == g["expect"]["self_mem_dep_at_use"]


def test_fig4a_predicate_coverage():
    g = load("fig4a_predicates.json")
    prog = assemble(g["program"])
    P = O.Program(prog)
    u = use_index(prog, g["use"]["instr"], loc(prog, g["use"]["loc"]))
    assert list(P.sources(u)) == g["expect"]["sources"]
    assert list(P.sources(u, blocked=True)) == g["expect"]["sources"]


def test_fig4c_opcode_pruning():
    g = load("fig4c_opcode_pruning.json")
    prog = assemble(g["program"])
    res = O.run_all(prog, recs(g["samples"]))
    bl = res["blame"]["blamed"]
    for i, v in g["expect"]["blamed_mem_dep_latency"].items():
        assert bl[int(i), S.ST_MEM_DEP, 1] == pytest.approx(v, rel=1e-15, abs=0)
    for i, v in g["expect"]["blamed_exec_dep_latency"].items():
        assert bl[int(i), S.ST_EXEC_DEP, 1] == pytest.approx(v, rel=1e-15, abs=0)


def test_fig4d_equal_apportioning():
    g = load("fig4d_apportion.json")
    prog = assemble(g["program"])
    res = O.run_all(prog, recs(g["samples"]))
    an = res["analysis"]
    for i, d in g["expect"]["dmax"].items():
        k = [t for t in range(an["n_edges"]) if an["src"][t] == int(i) and an["dst"][t] == 4]
        assert len(k) == 1 and an["dmax"][k[0]] == d
    bl = res["blame"]["blamed"]
    for i, v in g["expect"]["blamed_mem_dep_latency"].items():
        assert bl[int(i), S.ST_MEM_DEP, 1] == pytest.approx(v, rel=1e-15)


@pytest.mark.parametrize("case", [0, 1])
def test_theorem_latency_hiding_bound(case):
    g = load("theorem_bound.json")
    c = g["cases"][case]
    prog = assemble(g["program"])
    res = O.run_all(prog, recs(c["samples"]))
    est = res["estimate"]
    assert est["kernel_T"][0] == c["T"]
    assert est["kernel_L"][0] == c["L"]
    assert est["active"][0] == c["A"]
    for o in (S.OPTIMIZER_NAMES.index("LoopUnrolling"), S.OPTIMIZER_NAMES.index("CodeReordering")):
        assert est["matched"][0, o] == pytest.approx(c["ML"], rel=1e-15)
        assert est["speedup"][0, o] == pytest.approx(c["speedup"], rel=1e-15)
    # the loop scope holds both instructions: same matched samples and actives
    loop = int(np.nonzero(prog["scope_kind"] == S.SCOPE_LOOP)[0][0])
    lu = S.OPTIMIZER_NAMES.index("LoopUnrolling")
    assert est["matched"][loop, lu] == pytest.approx(c["ML"], rel=1e-15)
    assert est["speedup"][loop, lu] == pytest.approx(c["speedup"], rel=1e-15)


def test_load_use_chain_takes_all_stalls():
    """A straight-line load -> use chain with a single def: every memory
    dependency stall of the use goes to the load, even with no issued
    samples anywhere (Eq. 1 then apportions by path length alone)."""
    prog = assemble("block 0 ->\n  LDG R0 <- R2 R3\n  MOV R4 <- R5\n  IADD R1 <- R0 R4\n")
    rec = recs([[2, "MEM_DEP", 1, 4], [2, "MEM_DEP", 0, 3]])
    res = O.run_all(prog, rec)
    bl = res["blame"]
    assert bl["blamed"][0, S.ST_MEM_DEP].tolist() == [3.0, 4.0]
    assert bl["self"][2, S.ST_MEM_DEP].tolist() == [0.0, 0.0]
    assert bl["fine"][0, 0].tolist() == [3.0, 4.0]       # global-memory fine class


def test_dominator_pruning_hand_case():
    """LDG R0; MOV R5,R0; IADD R1,R0: the unpredicated MOV uses R0 on every
    path from the LDG to the IADD, so the LDG->IADD edge is pruned (Sec. 4,
    rule 2) while LDG->MOV is kept."""
    prog = assemble("block 0 ->\n  LDG R0 <- R2 R3\n  MOV R5 <- R0\n  IADD R1 <- R0\n")
    an = O.Program(prog).analyze()
    edges = {(int(s), int(d)): int(f) for s, d, f in zip(an["src"], an["dst"], an["flags"])}
    assert edges[(0, 2)] & 1 == 0
    assert edges[(0, 1)] & 1 == 1
    # a predicated MOV does not dominate: the edge survives
    prog2 = assemble("block 0 ->\n  LDG R0 <- R2 R3\n  @P1 MOV R5 <- R0\n  IADD R1 <- R0\n")
    an2 = O.Program(prog2).analyze()
    e2 = {(int(s), int(d)): int(f) for s, d, f in zip(an2["src"], an2["dst"], an2["flags"])}
    assert e2[(0, 2)] & 1 == 1


def test_latency_pruning_hand_case():
    """An ALU def (latency 6) reaching a use across 7 instructions is pruned
    by the latency rule (Sec. 4, rule 3); across 6 it is kept."""
    fill = "".join(f"  MOV R{8 + k} <- R15\n" for k in range(7))
    prog = assemble("block 0 ->\n  IADD R0 <- R1\n" + fill + "  IADD R2 <- R0\n")
    an = O.Program(prog).analyze()
    k = [t for t in range(an["n_edges"]) if an["src"][t] == 0 and an["dst"][t] == 8][0]
    assert an["dmin"][k] == 7 and (an["flags"][k] & 2) == 0
    fill6 = "".join(f"  MOV R{8 + k} <- R15\n" for k in range(6))
    prog = assemble("block 0 ->\n  IADD R0 <- R1\n" + fill6 + "  IADD R2 <- R0\n")
    an = O.Program(prog).analyze()
    k = [t for t in range(an["n_edges"]) if an["src"][t] == 0 and an["dst"][t] == 7][0]
    assert an["dmin"][k] == 6 and (an["flags"][k] & 2) == 2


def test_war_subclass():
    """A store reads its data register and sets a read barrier; the next
    writer of that register waits on it: a write-after-read execution
    dependency (Sec. 4, Fig. 5)."""
    prog = assemble("block 0 ->\n  STG <- R2 R3 R0 | rbar B1\n  MOV R0 <- R4 | wait B1\n")
    rec = recs([[1, "EXEC_DEP", 1, 5]])
    res = O.run_all(prog, rec)
    an = res["analysis"]
    assert list(zip(an["src"].tolist(), an["dst"].tolist())) == [(0, 1)]
    assert an["flags"][0] & 4
    assert res["blame"]["fine"][0, 5, 1] == 5.0        # EXEC_WAR


def test_eq2_stall_elimination_closed_form():
    prog = assemble("block 0 ->\n  IADD R1 <- R0\n  LDG R2 <- R4 R5\n")
    rec = recs([[0, "SELECTED", 0, 6], [1, "INST_FETCH", 1, 2], [1, "INST_FETCH", 0, 2],
                [1, "MEM_THROTTLE", 1, 3]])
    est = O.run_all(prog, rec)["estimate"]
    T = 13.0
    fs = S.OPTIMIZER_NAMES.index("FunctionSplit")
    mt = S.OPTIMIZER_NAMES.index("MemoryTransactionReduction")
    assert est["speedup"][0, fs] == T / (T - 4.0)
    assert est["speedup"][0, mt] == T / (T - 3.0)
    assert est["speedup"][0, 0] == 1.0          # nothing matched


def test_nested_scope_actives():
    """Eq. (5) and its example: loop2 holds loop1, so the active samples
    bounding loop2's estimate include loop1's."""
    prog = assemble("block 0 -> 1\n  IADD R1 <- R0\nblock 1 -> 1 2\n  IADD R2 <- R1\n  BRA\n"
                    "block 2 -> 0 3\n  MOV R3 <- R2\n  BRA\nblock 3 ->\n  MOV R4 <- R3\n"
                    "loop 0 2\nloop 1 1\n")
    rec = recs([[1, "SELECTED", 0, 2], [3, "SELECTED", 0, 3], [5, "SELECTED", 0, 7],
                [1, "MEM_DEP", 1, 4]])
    est = O.run_all(prog, rec)["estimate"]
    loops = np.nonzero(prog["scope_kind"] == S.SCOPE_LOOP)[0]
    outer, inner = int(loops[0]), int(loops[1])
    assert prog["scope_parent"][inner] == outer
    assert est["active"][inner] == 2 and est["active"][outer] == 5 and est["active"][0] == 12
