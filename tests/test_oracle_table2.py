"""Pins of the oracle's Table 2 matching rules, Fig. 5 fine classes, Eq. (3),
the ranking order and the saturated estimate against hand-worked programs
(tests/golden, each file citing its passage)."""
import json
import math
import os

import numpy as np
import pytest

from asm import assemble, samples
from oracle import oracle as O
from paper_2009_04061_amd import synth as S

GOLD = os.path.join(os.path.dirname(__file__), "golden")
FINE = ["MEM_GLOBAL", "MEM_LOCAL", "MEM_CONST", "EXEC_SHARED", "EXEC_ARITH", "EXEC_WAR", "SYNC",
        "OTHER"]
OPT = {name: k for k, name in enumerate(S.OPTIMIZER_NAMES)}


def load(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def recs(spec):
    return samples([(pc, S.STALL_NAMES.index(st), lam, n) for pc, st, lam, n in spec])


def run(g, spec=None):
    prog = assemble(g["program"])
    return prog, O.run_all(prog, recs(spec if spec is not None else g["samples"]), k=6)


def approx(v):
    return pytest.approx(v, rel=1e-14, abs=1e-14)


def scopes_where(prog, kind, flags=None):
    out = []
    for s in range(len(prog["scope_kind"])):
        if prog["scope_kind"][s] != kind:
            continue
        if flags is not None and (int(prog["scope_flags"][s]) & flags) != flags:
            continue
        out.append(s)
    return out


def test_register_reuse_and_memory_fine_classes():
    g = load("table2_register_reuse.json")
    prog, res = run(g)
    e = g["expect"]
    bl, fine = res["blame"]["blamed"], res["blame"]["fine"]
    for i, v in e["blamed_mem_dep"].items():
        assert bl[int(i), S.ST_MEM_DEP].tolist() == approx(v)
    for i, (cls, a, l) in e["fine"].items():
        f = FINE.index(cls)
        assert fine[int(i), f].tolist() == approx([a, l])
        # and nothing in any other fine class
        assert fine[int(i)].sum() == approx(a + l)
    est = res["estimate"]
    rr = OPT["RegisterReuse"]
    assert est["matched"][0, rr] == approx(e["matched"]["RegisterReuse"]["root"])
    for i, v in e["matched"]["RegisterReuse"]["line_of"].items():
        assert est["matched"][prog["instr_scope"][int(i)], rr] == approx(v)
    assert est["kernel_T"][0] == e["T"]
    num, den = e["speedup_root"]["RegisterReuse"]
    assert est["speedup"][0, rr] == approx(num / den)


def test_strength_reduction_and_execution_fine_classes():
    g = load("table2_strength_reduction.json")
    prog, res = run(g)
    e = g["expect"]
    bl, fine = res["blame"]["blamed"], res["blame"]["fine"]
    for i, v in e["blamed_exec_dep"].items():
        assert bl[int(i), S.ST_EXEC_DEP].tolist() == approx(v)
    for i, (cls, a, l) in e["fine"].items():
        assert fine[int(i), FINE.index(cls)].tolist() == approx([a, l])
        assert fine[int(i)].sum() == approx(a + l)
    est = res["estimate"]
    sr = OPT["StrengthReduction"]
    assert est["matched"][0, sr] == approx(e["matched"]["StrengthReduction"]["root"])
    for i, v in e["matched"]["StrengthReduction"]["line_of"].items():
        assert est["matched"][prog["instr_scope"][int(i)], sr] == approx(v)
    num, den = e["speedup_root"]["StrengthReduction"]
    assert est["speedup"][0, sr] == approx(num / den)


def test_fast_math_uses_the_math_flag_and_inlining_skips_inlined_scopes():
    g = load("table2_fast_math.json")
    prog, res = run(g)
    e = g["expect"]
    est = res["estimate"]
    assert est["kernel_T"][0] == e["T"]
    for name, v in e["matched_root"].items():
        assert est["matched"][0, OPT[name]] == approx(v)
    (math_fn,) = scopes_where(prog, S.SCOPE_FUNCTION, S.SF_MATH_FN)
    assert est["matched"][math_fn, OPT["FastMath"]] == approx(e["matched_math_fn"]["FastMath"])
    for name, (num, den) in e["speedup_root"].items():
        assert est["speedup"][0, OPT[name]] == approx(num / den)


def test_function_inlining_counts_latency_samples_of_called_device_functions():
    g = load("table2_function_inlining.json")
    prog, res = run(g)
    e = g["expect"]
    est = res["estimate"]
    fi = OPT["FunctionInlining"]
    (dev,) = [s for s in scopes_where(prog, S.SCOPE_FUNCTION, S.SF_DEVICE_FN | S.SF_HAS_CFG)]
    assert prog["scope_parent"][dev] == 0
    assert est["kernel_T"][0] == e["T"]
    assert est["active"][0] == e["A_root"] and est["active"][dev] == e["A_device_fn"]
    assert est["matched"][0, fi] == approx(e["matched_root"]["FunctionInlining"])
    assert est["matched"][dev, fi] == approx(e["matched_device_fn"]["FunctionInlining"])
    for i, v in e["matched_line_of"].items():
        assert est["matched"][prog["instr_scope"][int(i)], fi] == approx(v)
    num, den = e["speedup_root"]["FunctionInlining"]
    assert est["speedup"][0, fi] == approx(num / den)
    num, den = e["speedup_device_fn"]["FunctionInlining"]
    assert est["speedup"][dev, fi] == approx(num / den)


def test_warp_balance_takes_blamed_and_kept_synchronization_stalls():
    g = load("table2_warp_balance.json")
    prog, res = run(g)
    e = g["expect"]
    bl = res["blame"]
    for i, v in e["blamed_sync"].items():
        assert bl["blamed"][int(i), S.ST_SYNC].tolist() == approx(v)
    for i, v in e["self_sync"].items():
        assert bl["self"][int(i), S.ST_SYNC].tolist() == approx(v)
    est = res["estimate"]
    wb = OPT["WarpBalance"]
    for i, v in e["matched_line_of"].items():
        assert est["matched"][prog["instr_scope"][int(i)], wb] == approx(v)
    assert est["matched"][0, wb] == approx(e["matched_root"])
    num, den = e["speedup_root"]
    assert est["speedup"][0, wb] == approx(num / den)


def test_loop_unrolling_goes_to_the_innermost_common_loop():
    g = load("table2_loop_unrolling_target.json")
    prog, res = run(g)
    e = g["expect"]
    bl = res["blame"]["blamed"]
    for i, v in e["blamed_mem_dep"].items():
        assert bl[int(i), S.ST_MEM_DEP].tolist() == approx(v)
    (loop,) = scopes_where(prog, S.SCOPE_LOOP)
    (fn,) = scopes_where(prog, S.SCOPE_FUNCTION, S.SF_DEVICE_FN)
    assert prog["scope_parent"][fn] == loop
    est = res["estimate"]
    where = {"root": 0, "loop": loop, "inlined_fn": fn}
    for name in ("LoopUnrolling", "CodeReordering"):
        for key, s in where.items():
            assert est["matched"][s, OPT[name]] == approx(e[name][key]), (name, key)


def test_eq3_differs_from_eq4_when_active_samples_bound_the_hiding():
    g = load("theorem_bound.json")
    prog = assemble(g["program"])
    for c in g["cases"]:
        est = O.run_all(prog, recs(c["samples"]))["estimate"]
        for h, name in enumerate(("LoopUnrolling", "CodeReordering", "FunctionInlining")):
            assert est["eq3"][0, h] == approx(c["eq3"][name]), name


def test_ranking_ties_break_by_optimizer_then_scope():
    g = load("ranking_tie.json")
    prog, res = run(g)
    e = g["expect"]
    est = res["estimate"]
    top = list(zip(est["top_opt"][0].tolist(), est["top_scope"][0].tolist()))
    assert top == [tuple(t) for t in e["top"]]
    for got, (num, den) in zip(est["top_speed"][0].tolist(), e["top_speed"]):
        assert got == num / den


@pytest.mark.parametrize("case", [0, 1])
def test_saturated_estimate_is_infinite(case):
    g = load("saturated_estimate.json")
    c = g["cases"][case]
    prog = assemble(c["program"])
    est = O.run_all(prog, recs(c["samples"]))["estimate"]
    o = OPT[c["optimizer"]]
    assert est["kernel_T"][0] == c["T"]
    if c.get("matched_above_T"):
        assert est["matched"][0, o] > c["T"]
    assert est["speedup"][0, o] == math.inf
    # no estimate anywhere is negative or NaN
    sp = est["speedup"]
    assert not np.isnan(sp).any() and (sp >= 1.0).all()
