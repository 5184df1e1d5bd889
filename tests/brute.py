"""Brute-force definitions used to pin the oracle on tiny programs.

These are deliberately different computations from the oracle's:
  * sources: forward enumeration of simple walks from every def to the use,
    checking the kill rule at each intermediate position;
  * textbook reaching definitions (no guards): iterative gen/kill sets;
  * dmin: breadth-first search; dmax: enumeration of every walk in the CFG
    with its dominance back edges removed (for reducible CFGs these are the
    retreating edges of any depth-first search).
"""
from __future__ import annotations

import numpy as np

from paper_2009_04061_amd import synth as S


class Prog:
    def __init__(self, p):
        self.p = p
        self.n = len(p["op_class"])
        bb = p["block_begin"]
        self.nb = len(bb) - 1
        self.block_of = np.zeros(self.n, np.int64)
        for b in range(self.nb):
            self.block_of[bb[b]:bb[b + 1]] = b
        self.bsucc = [list(map(int, p["succ"][p["succ_ptr"][b]:p["succ_ptr"][b + 1]]))
                      for b in range(self.nb)]
        self.defs = [list(map(int, p["def_loc"][p["def_ptr"][k]:p["def_ptr"][k + 1]]))
                     for k in range(self.n)]
        self.dkind = [list(map(int, p["def_kind"][p["def_ptr"][k]:p["def_ptr"][k + 1]]))
                      for k in range(self.n)]
        self.uses = [list(map(int, p["use_loc"][p["use_ptr"][k]:p["use_ptr"][k + 1]]))
                     for k in range(self.n)]
        self.guard = list(map(int, p["guard"]))
        self.func_of_block = np.zeros(self.nb, np.int64)
        fbb = p["func_block_begin"]
        for f in range(len(fbb) - 1):
            self.func_of_block[fbb[f]:fbb[f + 1]] = f

    def first(self, b):
        return int(self.p["block_begin"][b])

    def last(self, b):
        return int(self.p["block_begin"][b + 1]) - 1

    def succ(self, k, skip_edges=frozenset()):
        b = int(self.block_of[k])
        if k < self.last(b):
            return [k + 1]
        return [self.first(s) for s in self.bsucc[b] if (b, s) not in skip_edges]

    def use_site(self, u):
        j = int(np.searchsorted(self.p["use_ptr"], u, side="right")) - 1
        x = int(self.p["use_loc"][u])
        c = self.guard[j] if int(self.p["use_kind"][u]) == S.USE_OPND else 0
        return j, x, c

    def partner(self, k, x):
        g = self.guard[k]
        if g == 0:
            return None
        comp = g + 1 if g % 2 == 1 else g - 1
        b = int(self.block_of[k])
        for q in range(k - 1, self.first(b) - 1, -1):
            if x in self.defs[q]:
                return q if self.guard[q] == comp else None
        return None


def kills(P: Prog, k, x, c, d, blocked):
    """Does intermediate position k stop def d of x from reaching the use?"""
    if x in P.defs[k]:
        if P.guard[k] == 0 or P.guard[k] == c:
            return True
        if P.partner(k, x) is not None and P.partner(k, x) != d:
            return True
    if blocked and P.guard[k] == 0 and x in P.uses[k]:
        return True
    return False


def src_brute(P: Prog, u, blocked):
    j, x, c = P.use_site(u)
    f = P.func_of_block[P.block_of[j]]
    out = []
    for d in range(P.n):
        if x not in P.defs[d] or P.func_of_block[P.block_of[d]] != f:
            continue
        # DFS over simple walks d -> ... -> j whose intermediates do not kill
        found = False
        stack = [(s, frozenset()) for s in P.succ(d)]
        seen_states = set()
        while stack and not found:
            v, path = stack.pop()
            if v == j:
                found = True
                break
            if v in path or kills(P, v, x, c, d, blocked):
                continue
            key = (v, path)
            if key in seen_states:
                continue
            seen_states.add(key)
            np_ = path | {v}
            for w in P.succ(v):
                stack.append((w, np_))
        if found:
            out.append(d)
    return out


def textbook_rd(P: Prog):
    """Classic reaching definitions for unguarded code: every def of x kills
    every other def of x.  Returns {use index: sorted def instructions}."""
    n = P.n
    preds = [[] for _ in range(n)]
    for k in range(n):
        for w in P.succ(k):
            preds[w].append(k)
    IN = [set() for _ in range(n)]
    OUT = [set() for _ in range(n)]
    changed = True
    while changed:
        changed = False
        for k in range(n):
            inn = set()
            for q in preds[k]:
                inn |= OUT[q]
            out = {(d, x) for (d, x) in inn if x not in P.defs[k]} | {(k, x) for x in P.defs[k]}
            if inn != IN[k] or out != OUT[k]:
                IN[k], OUT[k] = inn, out
                changed = True
    res = {}
    for u in range(int(P.p["use_ptr"][-1])):
        j, x, _ = P.use_site(u)
        res[u] = sorted(d for (d, y) in IN[j] if y == x)
    return res


def dmin_bfs(P: Prog, i, j):
    from collections import deque
    seen = set()
    q = deque()
    for s in P.succ(i):
        if s not in seen:
            seen.add(s)
            q.append((s, 1))
    while q:
        v, m = q.popleft()
        if v == j:
            return m - 1
        for w in P.succ(v):
            if w not in seen:
                seen.add(w)
                q.append((w, m + 1))
    return None


def dominance_back_edges(P: Prog, f):
    """Block edges u -> v of function f with v dominating u (every path from
    the entry to u passes v), by the definition: remove v, test reachability."""
    fbb = P.p["func_block_begin"]
    b0, b1 = int(fbb[f]), int(fbb[f + 1])

    def reach(removed):
        seen = set()
        if removed == b0:
            return seen
        st = [b0]
        while st:
            b = st.pop()
            if b in seen or b == removed:
                continue
            seen.add(b)
            st.extend(P.bsucc[b])
        return seen

    full = reach(None)
    back = set()
    for u in range(b0, b1):
        for v in P.bsucc[u]:
            if u in full and (v == u or u not in reach(v)):
                back.add((u, v))
    return back


def dmax_paths(P: Prog, i, j, back):
    """Maximum over all walks in the CFG minus `back` of the instructions
    strictly between i and j (None if no such walk)."""
    best = [None]

    def rec(v, m, onpath):
        if v == j:
            if best[0] is None or m - 1 > best[0]:
                best[0] = m - 1
            return
        for w in P.succ(v, back):
            if w in onpath:
                raise AssertionError("cycle left in G'")
            rec(w, m + 1, onpath | {w})

    for s in P.succ(i, back):
        rec(s, 1, frozenset({s}))
    return best[0]


# ------------------------------------------------------- random tiny programs
def random_cfg_program(seed, n_blocks=5, max_block=4, n_locs=3, n_preds=2, guard_p=0.35,
                       pair_p=0.3, reducible=False):
    """A random tiny program; with reducible=False the CFG is arbitrary
    (possibly irreducible, possibly with unreachable blocks)."""
    rng = np.random.default_rng(seed)
    if reducible:
        return S.gen_program(functions=[dict(n_instr=int(rng.integers(2 * n_blocks, 4 * n_blocks + 1)),
                                             n_blocks=n_blocks, n_loops=2, max_depth=2, kind="kernel")],
                             n_regs=n_locs, n_preds=n_preds, n_bars=2, guard_frac=guard_p,
                             pair_frac=pair_p, branch_frac=0.5, rng=rng)
    sizes = rng.integers(1, max_block + 1, size=n_blocks)
    n = int(sizes.sum())
    succ_lists = []
    for b in range(n_blocks):
        k = int(rng.integers(0, 3))
        succ_lists.append([int(t) for t in rng.integers(0, n_blocks, size=k)])
        succ_lists[-1] = list(dict.fromkeys(succ_lists[-1]))
    op, guard, defs, uses = [], [], [], []
    for k in range(n):
        g = 0
        if rng.random() < guard_p:
            g = S.guard_literal(int(rng.integers(n_preds)), bool(rng.random() < 0.5))
        d = []
        if rng.random() < 0.75:
            d.append((int(rng.integers(n_locs)), S.DEF_REG if rng.random() < 0.8 else S.DEF_RBAR))
        us = []
        for _ in range(int(rng.integers(0, 3))):
            us.append((int(rng.integers(n_locs)), S.USE_OPND if rng.random() < 0.7 else S.USE_WAIT))
        if g:
            us.append((n_locs + (g - 1) // 2, S.USE_GUARD))
        us = list(dict.fromkeys(us))
        # complementary pair on the same location right after a guarded def
        if k > 0 and rng.random() < pair_p and guard[-1] != 0 and defs[-1]:
            g = guard[-1] + 1 if guard[-1] % 2 == 1 else guard[-1] - 1
            d = [(defs[-1][0][0], S.DEF_REG)]
        op.append(int(rng.integers(0, 13)))
        guard.append(g)
        defs.append(d)
        uses.append(us)
    bb = np.zeros(n_blocks + 1, np.uint32)
    bb[1:] = np.cumsum(sizes)
    def_ptr = np.zeros(n + 1, np.uint32)
    def_ptr[1:] = np.cumsum([len(d) for d in defs])
    use_ptr = np.zeros(n + 1, np.uint32)
    use_ptr[1:] = np.cumsum([len(u) for u in uses])
    succ_ptr = np.zeros(n_blocks + 1, np.uint32)
    succ_ptr[1:] = np.cumsum([len(s) for s in succ_lists])
    arch = S.default_arch()
    return {
        "n_regs": n_locs, "n_preds": n_preds, "n_bars": 0,
        "op_class": np.array(op, np.uint8), "guard": np.array(guard, np.uint8),
        "def_ptr": def_ptr, "def_loc": np.array([l for d in defs for l, _ in d], np.uint32),
        "def_kind": np.array([kk for d in defs for _, kk in d], np.uint8),
        "use_ptr": use_ptr, "use_loc": np.array([l for u in uses for l, _ in u], np.uint32),
        "use_kind": np.array([kk for u in uses for _, kk in u], np.uint8),
        "block_begin": bb, "succ_ptr": succ_ptr,
        "succ": np.array([t for s in succ_lists for t in s], np.uint32),
        "func_block_begin": np.array([0, n_blocks], np.uint32),
        "func_scope": np.array([0], np.uint32),
        "instr_scope": np.arange(1, n + 1, dtype=np.uint32),
        "scope_parent": np.array([S.NO_PARENT] + [0] * n, np.uint32),
        "scope_kind": np.array([S.SCOPE_FUNCTION] + [S.SCOPE_LINE] * n, np.uint8),
        "scope_flags": np.array([S.SF_KERNEL_ENTRY | S.SF_HAS_CFG] + [0] * n, np.uint8),
        "lat": arch["lat"], "allowed": arch["allowed"], "blamable": int(arch["blamable"]),
    }
