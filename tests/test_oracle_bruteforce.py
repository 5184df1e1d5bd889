"""Pins of the oracle's exact steps against brute force on tiny programs and
against textbook special cases."""
import numpy as np
import pytest

import brute as B
from oracle import oracle as O
from paper_2009_04061_amd import synth as S


def _programs():
    for seed in range(40):
        yield ("arbitrary", seed), B.random_cfg_program(seed, n_blocks=5, max_block=4)
    for seed in range(25):
        yield ("structured", seed), B.random_cfg_program(1000 + seed, n_blocks=6, reducible=True)


PROGS = list(_programs())


@pytest.mark.parametrize("tag,prog", PROGS, ids=[f"{t[0]}-{t[1]}" for t, _ in PROGS])
def test_sources_match_simple_path_enumeration(tag, prog):
    P = O.Program(prog)
    BP = B.Prog(prog)
    for u in range(P.n_uses):
        for blocked in (False, True):
            got = P.sources(u, blocked).tolist()
            want = B.src_brute(BP, u, blocked)
            assert got == want, (u, blocked)


@pytest.mark.parametrize("seed", range(30))
def test_unguarded_code_is_textbook_reaching_definitions(seed):
    prog = B.random_cfg_program(500 + seed, n_blocks=6, max_block=5, guard_p=0.0, pair_p=0.0)
    assert not prog["guard"].any()
    P = O.Program(prog)
    want = B.textbook_rd(B.Prog(prog))
    for u in range(P.n_uses):
        assert P.sources(u).tolist() == want[u]


@pytest.mark.parametrize("seed", range(25))
def test_distances_match_bfs_and_path_enumeration(seed):
    prog = B.random_cfg_program(2000 + seed, n_blocks=7, reducible=True)
    P = O.Program(prog)
    BP = B.Prog(prog)
    back = B.dominance_back_edges(BP, 0)
    an = P.analyze()
    assert an["n_edges"] > 0
    for e in range(an["n_edges"]):
        i, j = int(an["src"][e]), int(an["dst"][e])
        assert an["dmin"][e] == B.dmin_bfs(BP, i, j)
        dm = B.dmax_paths(BP, i, j, back)
        assert an["dmax"][e] == (an["dmin"][e] if dm is None else dm)
        lat = prog["lat"][prog["op_class"][i]]
        assert bool(an["flags"][e] & 2) == (an["dmin"][e] <= lat)


@pytest.mark.parametrize("seed", range(20))
def test_distances_on_arbitrary_cfgs(seed):
    """Irreducible CFGs: dmin is still BFS; dmax is bounded below by dmin and
    is attained by a walk that never repeats an instruction."""
    prog = B.random_cfg_program(3000 + seed, n_blocks=6)
    P = O.Program(prog)
    BP = B.Prog(prog)
    an = P.analyze()
    for e in range(an["n_edges"]):
        i, j = int(an["src"][e]), int(an["dst"][e])
        assert an["dmin"][e] == B.dmin_bfs(BP, i, j)
        assert an["dmax"][e] >= an["dmin"][e]


def test_edge_table_is_union_of_sources():
    prog = B.random_cfg_program(77, n_blocks=8, reducible=True)
    P = O.Program(prog)
    an = P.analyze()
    edges = set(zip(an["src"].tolist(), an["dst"].tolist()))
    dom = {(int(s), int(d)) for s, d, f in zip(an["src"], an["dst"], an["flags"]) if f & 1}
    want, want_dom = set(), set()
    for u in range(P.n_uses):
        j = int(np.searchsorted(prog["use_ptr"], u, side="right")) - 1
        want |= {(int(i), j) for i in P.sources(u)}
        want_dom |= {(int(i), j) for i in P.sources(u, True)}
    assert edges == want and dom == want_dom
    # sorted by destination, then source
    key = an["dst"].astype(np.int64) * 10**6 + an["src"]
    assert (np.diff(key) > 0).all()


def test_counts_are_bincount_and_drop_invalid():
    prog, rec = S.workload_small(seed=3, n_samples=50_000)
    bad = S.corrupt_samples(rec, 0.02, 2000, seed=4)
    C, dropped = O.count(2000, bad)
    valid = (bad["pc"] < 2000) & (bad["stall"] < 12) & ((bad["flags"] & 0xFE) == 0) & (bad["reserved"] == 0)
    key = (bad["pc"][valid].astype(np.int64) * 12 + bad["stall"][valid]) * 2 + (bad["flags"][valid] & 1)
    assert (C.reshape(-1) == np.bincount(key, minlength=2000 * 24)).all()
    assert dropped == int((~valid).sum()) and dropped > 0
    assert C.sum() == valid.sum()


def test_empty_profile():
    prog, _ = S.workload_small(seed=0, n_samples=10)
    res = O.run_all(prog, np.zeros(0, S.SAMPLE_DTYPE))
    assert res["C"].sum() == 0 and res["dropped"] == 0
    assert (res["estimate"]["speedup"] == 1.0).all()
    assert res["blame"]["share"].sum() == 0


@pytest.mark.parametrize("maker", ["small", "multi"])
def test_conservation_and_estimator_invariants(maker):
    prog, rec = (S.workload_small(seed=2, n_samples=100_000) if maker == "small"
                 else S.workload_multi(seed=7, n_samples=120_000))
    res = O.run_all(prog, rec)
    C, bl, est = res["C"].astype(np.float64), res["blame"], res["estimate"]
    nbl = bin(prog["blamable"]).count("1")
    assert bl["share"].shape[1] == nbl
    # conservation: blamed shares plus retained samples equal the samples, per reason and bit
    slot = 0
    for r in range(12):
        for lam in range(2):
            tot = C[:, r, lam].sum()
            kept = bl["self"][:, r, lam].sum()
            if (prog["blamable"] >> r) & 1:
                moved = bl["share"][:, slot, lam].sum()
                assert np.isclose(moved + kept, tot, rtol=1e-12, atol=0)
                assert np.isclose(bl["blamed"][:, r, lam].sum(), moved, rtol=1e-12)
            else:
                assert kept == tot and bl["blamed"][:, r, lam].sum() == 0
        if (prog["blamable"] >> r) & 1:
            slot += 1
    assert np.isclose(bl["fine"].sum(), bl["blamed"].sum(), rtol=1e-12)
    # T = A + L per kernel, Sec. 2.1
    roots = np.nonzero(prog["scope_parent"] == S.NO_PARENT)[0]
    for r in roots:
        assert est["kernel_T"][r] == est["active"][r] + est["kernel_L"][r]
    sp = est["speedup"]
    assert (sp[:, :6] >= 1.0).all()
    assert (sp[:, 6:] >= 1.0).all() and (sp[:, 6:] <= 2.0 + 1e-12).all()   # the theorem
    # subtree sums only grow towards the root, so do the estimates
    par = prog["scope_parent"]
    for s in range(len(par)):
        if par[s] != S.NO_PARENT:
            assert (est["matched"][par[s]] >= est["matched"][s] - 1e-9).all()
            assert (sp[par[s]] >= sp[s] - 1e-12).all()
            assert est["active"][par[s]] >= est["active"][s]
    # top-k ordering
    for r in roots:
        v = est["top_speed"][r]
        assert (np.diff(v) <= 0).all()
        assert v[0] == sp[est["root_of"] == r].max()
