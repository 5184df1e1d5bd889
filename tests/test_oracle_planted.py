"""Planted mistakes: the pins must catch plausible errors in the oracle.

Each case copies the oracle's C source, turns one expression into a plausible
mistake (a dropped rule, a wrong sign, index or bound, a transposed operand),
compiles the copy with the oracle's flags and reruns the pins chosen to catch
it; at least one of them must fail.  The committed oracle is never touched:
the copy lives in a temporary directory and is loaded only inside the test.
"""
import os

import pytest

import test_oracle_bruteforce as TB
import test_oracle_parallel as TP
import test_oracle_report as TR
import test_oracle_table2 as T2
import test_oracle_worked_examples as TW
from oracle import oracle as O

SRC = os.path.join(os.path.dirname(O.__file__), "gpa_oracle.c")


def _pins_for_sources():
    for tag, prog in TB.PROGS[::5]:
        TB.test_sources_match_simple_path_enumeration(tag, prog)


def _pins_for_distances():
    for seed in range(0, 25, 3):
        TB.test_distances_match_bfs_and_path_enumeration(seed)


# (name, original text, planted text, pins expected to catch it)
MUTANTS = [
    ("latency bit swapped in counting",
     "C[((size_t)pc * 12 + stall) * 2 + (flags & 1u)] += 1;",
     "C[((size_t)pc * 12 + stall) * 2 + (1u - (flags & 1u))] += 1;",
     [TB.test_counts_are_bincount_and_drop_invalid, TW.test_fig1_sampling_ratios]),
    ("reserved field not checked",
     "(flags & ~1u) == 0 && reserved == 0)",
     "(flags & ~1u) == 0)",
     [TB.test_counts_are_bincount_and_drop_invalid]),
    ("coverage ignores a matching guard",
     "static int covers(uint8_t g, uint8_t c) { return g == 0 || g == c; }",
     "static int covers(uint8_t g, uint8_t c) { return g == 0; }",
     [_pins_for_sources]),
    ("complementary pair rule dropped",
     "if (partner >= 0) {",
     "if (0 && partner >= 0) {",
     [TW.test_fig4a_predicate_coverage]),
    ("dominator stop also at predicated uses",
     "if (blocked && p->guard[k] == 0 && uses_loc(p, k, x)) continue;",
     "if (blocked && uses_loc(p, k, x)) continue;",
     [TW.test_dominator_pruning_hand_case, _pins_for_sources]),
    ("shortest distance counts an endpoint",
     "dmin[t] = d - 1;",
     "dmin[t] = d;",
     [TW.test_latency_pruning_hand_case, _pins_for_distances]),
    ("longest path keeps retreating edges",
     "        if (c->retreat[e]) continue;\n",
     "",
     [_pins_for_distances]),
    ("latency rule off by one",
     "if (d0[k - k0] <= p->lat[p->op_class[i]])",
     "if (d0[k - k0] < p->lat[p->op_class[i]])",
     [TW.test_latency_pruning_hand_case]),
    ("Eq. 1 path weight inverted",
     "issued / ((double)a->e_dmax[e] + 1.0)",
     "issued * ((double)a->e_dmax[e] + 1.0)",
     [TW.test_fig4d_equal_apportioning]),
    ("share credited to the destination",
     "blamed[((size_t)i * 12 + r) * 2 + l] += s;",
     "blamed[((size_t)j * 12 + r) * 2 + l] += s;",
     [TW.test_load_use_chain_takes_all_stalls, TW.test_fig3_barrier_dependency]),
    ("active and latency samples swapped",
     "      act += CNT(j, r, 0);\n      lat += CNT(j, r, 1);",
     "      act += CNT(j, r, 1);\n      lat += CNT(j, r, 0);",
     # Fig. 1 alone cannot see this one: its example has A = L = 3
     [TW.test_nested_scope_actives, lambda: TW.test_theorem_latency_hiding_bound(1)]),
    ("Eq. 5 without the active-sample bound",
     "double x = (o >= ORC_O_LOOP_UNROLL) ? (active[s] < M ? active[s] : M) : M;",
     "double x = M;",
     [lambda: TW.test_theorem_latency_hiding_bound(1)]),
    ("Eq. 2 sign",
     "double sp = (T == 0.0) ? 1.0 : (x >= T ? INFINITY : T / (T - x));",
     "double sp = (T == 0.0) ? 1.0 : (x >= T ? INFINITY : T / (T + x));",
     [TW.test_eq2_stall_elimination_closed_form]),
    ("subtree sums stop at the scope itself",
     "    if (p->scope_parent[s] == ORC_NONE) return;\n    s = p->scope_parent[s];",
     "    return;",
     [TW.test_nested_scope_actives]),
    # Table 2 matching rules
    ("Register Reuse matches global instead of local memory sources",
     "if (cls == ORC_LOCAL_LOAD || cls == ORC_LOCAL_STORE)\n      add_up(p, matched, ORC_N_OPT, ORC_O_REG_REUSE",
     "if (cls == ORC_GLOBAL_LOAD)\n      add_up(p, matched, ORC_N_OPT, ORC_O_REG_REUSE",
     [T2.test_register_reuse_and_memory_fine_classes]),
    ("Strength Reduction matches plain ALU sources",
     "if (cls == ORC_FP64 || cls == ORC_LONG_ALU)",
     "if (cls == ORC_ALU)",
     [T2.test_strength_reduction_and_execution_fine_classes]),
    ("Fast Math keyed on the device-function flag",
     "if (in_function_with(p, s, ORC_SF_MATH)) {",
     "if (in_function_with(p, s, ORC_SF_DEVICE)) {",
     [T2.test_fast_math_uses_the_math_flag_and_inlining_skips_inlined_scopes]),
    ("Warp Balance without the kept synchronization stalls",
     " +\n               self_[((size_t)j * 12 + ORC_SYNC) * 2] + self_[((size_t)j * 12 + ORC_SYNC) * 2 + 1]);",
     ");",
     [T2.test_warp_balance_takes_blamed_and_kept_synchronization_stalls]),
    ("Function Inlining counts active instead of latency samples",
     "for (uint32_t r = 0; r < 12; ++r) v += CNT(j, r, 1);",
     "for (uint32_t r = 0; r < 12; ++r) v += CNT(j, r, 0);",
     [T2.test_function_inlining_counts_latency_samples_of_called_device_functions]),
    ("Function Inlining also matches inlined device-function scopes",
     "in_function_with(p, s, ORC_SF_DEVICE | ORC_SF_CFG)",
     "in_function_with(p, s, ORC_SF_DEVICE)",
     [T2.test_fast_math_uses_the_math_flag_and_inlining_skips_inlined_scopes]),
    ("Loop Unrolling target taken as the lowest common scope",
     "uint32_t loop = common_loop(p, si, sj, fscope);",
     "uint32_t loop = lca(p, si, sj);",
     [T2.test_loop_unrolling_goes_to_the_innermost_common_loop]),
    # Fig. 5 fine classes
    ("constant-memory sources put in the local fine class",
     "if (cls == ORC_CONST_LOAD) return ORC_F_MEM_CONST;",
     "if (cls == ORC_CONST_LOAD) return ORC_F_MEM_LOCAL;",
     [T2.test_register_reuse_and_memory_fine_classes]),
    ("shared-memory sources put in the arithmetic fine class",
     "if (cls == ORC_SHARED_LOAD) return ORC_F_EXEC_SHARED;",
     "if (cls == ORC_SHARED_LOAD) return ORC_F_EXEC_ARITH;",
     [T2.test_strength_reduction_and_execution_fine_classes]),
    # Eq. (3), ranking, saturation
    ("Eq. 3 bounded by the active samples like Eq. 4",
     "eq3[(size_t)s * 3 + h] = (T == 0.0) ? 1.0 : (M >= T ? INFINITY : T / (T - M));",
     "eq3[(size_t)s * 3 + h] = (T == 0.0) ? 1.0 : T / (T - (active[s] < M ? active[s] : M));",
     [T2.test_eq3_differs_from_eq4_when_active_samples_bound_the_hiding]),
    ("ranking ties broken by optimizer descending",
     "if (x->opt != y->opt) return x->opt < y->opt ? -1 : 1;",
     "if (x->opt != y->opt) return x->opt > y->opt ? -1 : 1;",
     [T2.test_ranking_ties_break_by_optimizer_then_scope]),
    ("ranking ties broken by scope descending",
     "return (x->scope > y->scope) - (x->scope < y->scope);",
     "return (x->scope < y->scope) - (x->scope > y->scope);",
     [T2.test_ranking_ties_break_by_optimizer_then_scope]),
    # parallel optimizers (Sec. 5.2, Eqs. (6)-(10))
    ("Eq. 8 with the issued ratio in place of its complement",
     "static double orc_issue(double r, double w) { return 1.0 - pow(1.0 - r, w); }",
     "static double orc_issue(double r, double w) { return 1.0 - pow(r, w); }",
     [lambda: TP.test_parallel_estimators_hand_worked(0)]),
    ("Eq. 10 multiplied by C_W instead of divided",
     "(1.0 / C_W) * C_I * f : 1.0;",
     "C_W * C_I * f : 1.0;",
     [lambda: TP.test_parallel_estimators_hand_worked(0)]),
    ("resident blocks not bounded by the grid's share",
     "uint64_t resident = per_sm < grid_share ? per_sm : grid_share;",
     "uint64_t resident = per_sm;",
     [lambda: TP.test_parallel_estimators_hand_worked(0)]),
    ("contention stalls without the not-selected samples",
     "if (r == ORC_PIPE_BUSY || r == ORC_MEM_THROTTLE || r == ORC_NOT_SELECTED) contention += v;",
     "if (r == ORC_PIPE_BUSY || r == ORC_MEM_THROTTLE) contention += v;",
     [lambda: TP.test_parallel_estimators_hand_worked(1)]),
    ("Thread Increase without its factor",
     "      f = W > 0.0 ? W_new / W : 1.0;",
     "      f = 1.0;",
     [lambda: TP.test_parallel_estimators_hand_worked(2)]),
    ("Thread Increase matched whatever limits residency",
     "matched = lim_blocks < other && resident == lim_blocks && warps_now < max_warps;",
     "matched = resident == lim_blocks && warps_now < max_warps;",
     [lambda: TP.test_parallel_estimators_hand_worked(3)]),
    # report layer (Sec. 6 coverage, Sec. 7 hotspots)
    ("coverage after pruning ignores the latency rule",
     "if (a->e_src[e] == a->rd_src[q] && (a->e_flags[e] & ORC_E_LAT_KEEP)) ++kept;",
     "if (a->e_src[e] == a->rd_src[q]) ++kept;",
     [TR.test_single_dependency_coverage_before_and_after_pruning]),
    ("hotspots ranked smallest first",
     "if (a->v != b->v) return a->v > b->v ? -1 : 1;",
     "if (a->v != b->v) return a->v < b->v ? -1 : 1;",
     [lambda: TR.test_hotspots_hand_worked(1)]),
    ("Loop Unrolling hotspots outside any common loop",
     "        if (common_loop(p, p->instr_scope[i], p->instr_scope[j], fscope) == ORC_NONE) v = 0.0;\n",
     "",
     [lambda: TR.test_hotspots_hand_worked(3)]),
    ("saturated estimate left to the plain formula",
     "double sp = (T == 0.0) ? 1.0 : (x >= T ? INFINITY : T / (T - x));",
     "double sp = (T == 0.0) ? 1.0 : T / (T - x);",
     [lambda: T2.test_saturated_estimate_is_infinite(1)]),
]


def test_every_planted_text_is_in_the_oracle():
    with open(SRC) as f:
        src = f.read()
    for name, old, _, _ in MUTANTS:
        assert src.count(old) >= 1, name


@pytest.mark.parametrize("case", range(len(MUTANTS)), ids=[m[0] for m in MUTANTS])
def test_pins_catch_planted_mistake(case, tmp_path):
    name, old, new, pins = MUTANTS[case]
    with open(SRC) as f:
        src = f.read()
    assert old in src
    lib = O.build_variant(src.replace(old, new), str(tmp_path / "libmutant.so"))
    caught = []
    with O.use_library(lib):
        for pin in pins:
            try:
                pin()
            except AssertionError:
                caught.append(getattr(pin, "__name__", "pin"))
    assert caught, f"no pin caught the planted mistake: {name}"
