"""Seeded synthetic programs and PC-sample records for the GPA hot path.

This module only *generates inputs*. It holds none of the method's
arithmetic (no counting, dataflow, blame or estimates), so that the HIP
library and the CPU oracle can both read the bytes it writes.

Data model (the paper's instruction model, Sec. 2.2 and Table 1):
  * an instruction has an opcode class, a guard literal (``_``, ``Pk`` or
    ``!Pk``), a list of defined locations and a list of used locations;
  * locations are registers ``R0..``, predicates ``P0..`` and the virtual
    barrier registers ``B0..`` (Sec. 4, "virtual barrier registers"): a
    write/read barrier association is a def, a wait mask is a use;
  * instructions form basic blocks, blocks form one CFG per function;
  * a scope tree (function / loop / line) carries the program structure the
    static analyzer recovers (Sec. 3, "Program structure").
A PC sample is 8 bytes: ``u32 pc, u8 stall, u8 flags, u16 reserved`` with
flags bit 0 set for a latency sample (Sec. 2.1: the scheduler issued
nothing when the sample was taken).
"""
from __future__ import annotations

import bisect

import numpy as np

# ---------------------------------------------------------------- encodings
OP_ALU, OP_FP64, OP_LONG_ALU, OP_GLOBAL_LOAD, OP_SHARED_LOAD, OP_LOCAL_LOAD, \
    OP_CONST_LOAD, OP_GLOBAL_STORE, OP_SHARED_STORE, OP_LOCAL_STORE, \
    OP_BRANCH, OP_BARRIER, OP_CALL = range(13)
N_OP_CLASSES = 13
OP_NAMES = ["ALU", "FP64", "LONG_ALU", "GLOBAL_LOAD", "SHARED_LOAD", "LOCAL_LOAD",
            "CONST_LOAD", "GLOBAL_STORE", "SHARED_STORE", "LOCAL_STORE",
            "BRANCH", "BARRIER", "CALL"]

ST_SELECTED, ST_INST_FETCH, ST_EXEC_DEP, ST_MEM_DEP, ST_TEXTURE, ST_SYNC, \
    ST_CONST_MEM_DEP, ST_PIPE_BUSY, ST_MEM_THROTTLE, ST_NOT_SELECTED, \
    ST_OTHER, ST_SLEEPING = range(12)
N_STALLS = 12
STALL_NAMES = ["SELECTED", "INST_FETCH", "EXEC_DEP", "MEM_DEP", "TEXTURE", "SYNC",
               "CONST_MEM_DEP", "PIPE_BUSY", "MEM_THROTTLE", "NOT_SELECTED",
               "OTHER", "SLEEPING"]

DEF_REG, DEF_PRED, DEF_WBAR, DEF_RBAR = range(4)
USE_OPND, USE_GUARD, USE_WAIT = range(3)

SCOPE_FUNCTION, SCOPE_LOOP, SCOPE_LINE = range(3)
SF_KERNEL_ENTRY, SF_DEVICE_FN, SF_MATH_FN, SF_HAS_CFG = 1, 2, 4, 8
NO_PARENT = 0xFFFFFFFF

SAMPLE_DTYPE = np.dtype([("pc", "<u4"), ("stall", "u1"), ("flags", "u1"),
                         ("reserved", "<u2")])
assert SAMPLE_DTYPE.itemsize == 8

OPTIMIZER_NAMES = ["RegisterReuse", "StrengthReduction", "FunctionSplit", "FastMath",
                   "WarpBalance", "MemoryTransactionReduction", "LoopUnrolling",
                   "CodeReordering", "FunctionInlining"]


def guard_literal(pred: int, negated: bool) -> int:
    """Guard byte of ``Pk`` (1 + 2k) or ``!Pk`` (2 + 2k); 0 is ``_``."""
    return 1 + 2 * pred + (1 if negated else 0)


def default_arch() -> dict:
    """Architecture table passed to both sides as an input.

    Latencies are in instruction slots and are arbitrary builder defaults,
    not measurements; global and local loads use a large upper bound in the
    spirit of the TLB-miss bound of Sec. 4 ("Instruction latency based
    pruning"). ``allowed[r]`` is a bitmask of opcode classes that may be
    blamed for stall reason ``r`` (Sec. 4, opcode based pruning: memory
    dependency stalls go to memory instructions, synchronization stalls to
    synchronization instructions; no rule is stated for execution
    dependency, so every class is allowed).
    """
    lat = np.zeros(16, np.uint16)
    lat[OP_ALU] = 6
    lat[OP_FP64] = 16
    lat[OP_LONG_ALU] = 32
    lat[OP_GLOBAL_LOAD] = 1024
    lat[OP_SHARED_LOAD] = 64
    lat[OP_LOCAL_LOAD] = 1024
    lat[OP_CONST_LOAD] = 256
    lat[OP_GLOBAL_STORE] = lat[OP_SHARED_STORE] = lat[OP_LOCAL_STORE] = 64
    lat[OP_BRANCH] = 8
    lat[OP_BARRIER] = 32
    lat[OP_CALL] = 32
    allowed = np.zeros(12, np.uint16)
    allowed[ST_MEM_DEP] = (1 << OP_GLOBAL_LOAD) | (1 << OP_LOCAL_LOAD) | (1 << OP_CONST_LOAD)
    allowed[ST_SYNC] = 1 << OP_BARRIER
    allowed[ST_EXEC_DEP] = (1 << N_OP_CLASSES) - 1
    blamable = (1 << ST_MEM_DEP) | (1 << ST_EXEC_DEP) | (1 << ST_SYNC)
    return {"lat": lat, "allowed": allowed, "blamable": np.uint16(blamable)}


# opcode mix of the plain-path workloads
BASE_OP_MIX = {OP_GLOBAL_LOAD: 0.15, OP_SHARED_LOAD: 0.10, OP_ALU: 0.50, OP_FP64: 0.05,
               OP_BRANCH: 0.08, OP_BARRIER: 0.02, OP_GLOBAL_STORE: 0.10}


def stall_mix_small() -> np.ndarray:
    m = np.full(N_STALLS, 0.025)
    m[ST_MEM_DEP] = 0.35
    m[ST_EXEC_DEP] = 0.25
    m[ST_SYNC] = 0.10
    m[ST_NOT_SELECTED] = 0.10
    return m / m.sum()


def stall_mix_memory_skewed() -> np.ndarray:
    m = stall_mix_small() * (0.5 / 0.65)
    m[ST_MEM_DEP] = 0.5
    return m / m.sum()


def _mix_array(mix: dict) -> np.ndarray:
    p = np.zeros(N_OP_CLASSES)
    for k, v in mix.items():
        p[k] = v
    return p / p.sum()


# ------------------------------------------------------------- CFG skeleton
def _gen_loops(rng, nb, n_loops, max_depth, one_nest_depth=None):
    """Properly nested loop intervals [header, latch] over block indices."""
    loops = []
    if one_nest_depth:
        # one nest of the given depth over random block ranges
        pts = np.sort(rng.choice(np.arange(nb - 1), size=2 * one_nest_depth, replace=False))
        for d in range(one_nest_depth):
            loops.append((int(pts[d]), int(pts[2 * one_nest_depth - 1 - d])))
        return loops
    attempts = 0
    while len(loops) < n_loops and attempts < 200 * max(n_loops, 1):
        attempts += 1
        length = int(min(nb - 1, max(2, rng.geometric(1.0 / 12.0) + 1)))
        h = int(rng.integers(0, nb - length)) if nb - length > 0 else 0
        t = h + length - 1
        if t <= h or t >= nb - 1:
            continue
        ok = True
        depth = 1
        for (a, b) in loops:
            disjoint = t < a or h > b
            inside = a < h and t < b
            outside = h < a and b < t
            if not (disjoint or inside or outside):
                ok = False
                break
            if a == h or b == t:
                ok = False
                break
            if inside:
                depth += 1
        if not ok:
            continue
        # depth of loops this one would enclose must stay bounded too
        for (a, b) in loops:
            if h < a and b < t:
                d_in = 1 + sum(1 for (c, e) in loops if c < a and b < e)
                if d_in + 1 > max_depth:
                    ok = False
                    break
        if ok and depth <= max_depth:
            loops.append((h, t))
    return loops


def _build_cfg(rng, nb, loops, branch_frac):
    """Successor lists for a structured CFG: fall-through, do-while back
    edges, if-then and if-then-else diamonds that stay within one loop level."""
    loopset = [frozenset(i for i, (h, t) in enumerate(loops) if h <= b <= t) for b in range(nb)]
    latch = {t for (_, t) in loops}
    header = {h for (h, _) in loops}
    kind = ["ft"] * nb          # ft | cond | jump | exit
    target = [None] * nb
    used = np.zeros(nb, bool)
    order = rng.permutation(nb)
    for b in order:
        b = int(b)
        if rng.random() >= branch_frac:
            continue
        ite = rng.random() < 0.5
        span = 4 if ite else 3
        if b + span - 1 > nb - 1:
            continue
        blocks = list(range(b, b + span))
        inner = blocks[:-1] if ite else blocks
        if any(used[x] for x in inner):
            continue
        if any(x in latch for x in inner) or any(x in header for x in blocks[1:]):
            continue
        if any(loopset[x] != loopset[b] for x in blocks):
            continue
        if ite:
            kind[b], target[b] = "cond", b + 2
            kind[b + 1], target[b + 1] = "jump", b + 3
            used[b:b + 3] = True
        else:
            kind[b], target[b] = "cond", b + 2
            used[b:b + 2] = True
    succs = []
    for b in range(nb):
        s = []
        if b in latch:
            h = [hh for (hh, tt) in loops if tt == b][0]
            s = [h, b + 1] if b + 1 < nb else [h]
            kind[b] = "cond"
        elif kind[b] == "cond":
            s = [target[b], b + 1]
        elif kind[b] == "jump":
            s = [target[b]]
        elif b + 1 < nb:
            s = [b + 1]
        else:
            kind[b] = "exit"
        if len(s) == 2 and rng.random() < 0.5:
            s = s[::-1]
        succs.append(s)
    return succs, kind


# ------------------------------------------------------------ instructions
class _Uniform:
    """Uniform draws taken from the generator in blocks (one numpy call per
    block instead of one per decision)."""

    def __init__(self, rng, block=1 << 16):
        self.rng, self.block = rng, block
        self.buf, self.i = [], 0

    def u(self):
        if self.i == len(self.buf):
            self.buf, self.i = self.rng.random(self.block).tolist(), 0
        v = self.buf[self.i]
        self.i += 1
        return v

    def below(self, k):
        """An integer uniform in [0, k)."""
        return min(int(self.u() * k), k - 1)


class _Emitter:
    """Accumulates one function's instructions, defs and uses."""

    def __init__(self, rng, n_regs, n_preds, n_bars):
        self.rng = rng
        self.U = _Uniform(rng)
        self.n_regs, self.n_preds, self.n_bars = n_regs, n_preds, n_bars
        self.op, self.guard = [], []
        self.defs, self.uses = [], []
        self.def_regs, self.def_reg_set = [], set()
        self.def_preds, self.def_pred_set = [], set()
        self.pending_load = {}     # register -> barrier awaited by its first reader
        self.pending_store = {}    # data register -> read barrier awaited by its next writer
        self.pending_bar = None    # barrier the next instruction waits on

    # location ids
    def preg(self, k):
        return self.n_regs + k

    def bar(self, k):
        return self.n_regs + self.n_preds + k

    def pick_reg(self):
        if self.def_regs:
            return self.def_regs[self.U.below(len(self.def_regs))]
        return self.U.below(self.n_regs)      # live-in

    def pick_pred(self):
        if self.def_preds:
            return self.def_preds[self.U.below(len(self.def_preds))]
        return self.U.below(self.n_preds)

    def emit(self, op, guard, def_regs=(), def_pred=None, use_regs=(), use_preds=(),
             wbar=None, rbar=None, guard_use=None):
        defs, uses = [], []
        seen_u = set()

        def add_use(loc, kind):
            if (loc, kind) not in seen_u:
                seen_u.add((loc, kind))
                uses.append((loc, kind))

        if self.pending_bar is not None:
            add_use(self.bar(self.pending_bar), USE_WAIT)
            self.pending_bar = None
        if guard_use is not None:
            add_use(self.preg(guard_use), USE_GUARD)
        for r in use_regs:
            add_use(r, USE_OPND)
            if r in self.pending_load:
                add_use(self.bar(self.pending_load.pop(r)), USE_WAIT)
        for p in use_preds:
            add_use(self.preg(p), USE_OPND)
        for r in def_regs:
            if r in self.pending_store:
                add_use(self.bar(self.pending_store.pop(r)), USE_WAIT)
            self.pending_load.pop(r, None)
            defs.append((r, DEF_REG))
            if r not in self.def_reg_set:
                self.def_reg_set.add(r)
                self.def_regs.append(r)
        if def_pred is not None:
            defs.append((self.preg(def_pred), DEF_PRED))
            if def_pred not in self.def_pred_set:
                self.def_pred_set.add(def_pred)
                self.def_preds.append(def_pred)
        if wbar is not None:
            defs.append((self.bar(wbar), DEF_WBAR))
        if rbar is not None:
            defs.append((self.bar(rbar), DEF_RBAR))
        self.op.append(op)
        self.guard.append(guard)
        self.defs.append(defs)
        self.uses.append(uses)
        return len(self.op) - 1


def _gen_function_body(rng, em: _Emitter, block_sizes, kind, op_mix, guard_frac, pair_frac,
                       pred_def_frac=0.12):
    p = _mix_array(op_mix)
    cdf = np.cumsum(p)
    cdf[-1] = 1.0
    cdf = cdf.tolist()
    U = em.U
    n_regs, n_preds, n_bars = em.n_regs, em.n_preds, em.n_bars
    for b, size in enumerate(block_sizes):
        forced_pair = None           # (register, guard) of a pending complementary def
        for k in range(size):
            last = k == size - 1
            if last and kind[b] in ("cond", "jump"):
                if kind[b] == "cond":
                    pk = em.pick_pred()
                    g = guard_literal(pk, U.u() < 0.5)
                    em.emit(OP_BRANCH, g, guard_use=pk)
                else:
                    em.emit(OP_BRANCH, 0)
                forced_pair = None
                continue
            if forced_pair is not None:
                r, g = forced_pair
                forced_pair = None
                em.emit(OP_ALU, g, def_regs=[r], use_regs=[em.pick_reg()],
                        guard_use=(g - 1) // 2)
                continue
            op = min(bisect.bisect_right(cdf, U.u()), N_OP_CLASSES - 1)
            g = 0
            gpred = None
            if U.u() < guard_frac:
                gpred = U.below(n_preds)
                g = guard_literal(gpred, U.u() < 0.5)
            if op == OP_ALU:
                if U.u() < pred_def_frac:
                    em.emit(op, g, def_pred=U.below(n_preds),
                            use_regs=[em.pick_reg(), em.pick_reg()], guard_use=gpred)
                else:
                    r = U.below(n_regs)
                    # a complementary-guarded redefinition right after this one
                    room = (k + 1 < size - 1) or (k + 1 < size and kind[b] not in ("cond", "jump"))
                    if room and U.u() < pair_frac:
                        if g == 0:
                            gpred = U.below(n_preds)
                            g = guard_literal(gpred, U.u() < 0.5)
                        comp = g + 1 if g % 2 == 1 else g - 1
                        forced_pair = (r, comp)
                    em.emit(op, g, def_regs=[r], use_regs=[em.pick_reg(), em.pick_reg()],
                            guard_use=gpred)
            elif op == OP_FP64:
                r = 2 * U.below(n_regs // 2)
                em.emit(op, g, def_regs=[r, r + 1], use_regs=[em.pick_reg(), em.pick_reg()],
                        guard_use=gpred)
            elif op == OP_LONG_ALU:
                em.emit(op, g, def_regs=[U.below(n_regs)], use_regs=[em.pick_reg()],
                        guard_use=gpred)
            elif op in (OP_GLOBAL_LOAD, OP_SHARED_LOAD, OP_LOCAL_LOAD, OP_CONST_LOAD):
                if op == OP_GLOBAL_LOAD and U.u() < 0.25:
                    r = 2 * U.below(n_regs // 2)
                    dr = [r, r + 1]
                else:
                    dr = [U.below(n_regs)]
                ur = [em.pick_reg(), em.pick_reg()] if op == OP_GLOBAL_LOAD else [em.pick_reg()]
                wb = U.below(n_bars)
                em.emit(op, g, def_regs=dr, use_regs=ur, wbar=wb, guard_use=gpred)
                for r in dr:
                    em.pending_load[r] = wb
            elif op in (OP_GLOBAL_STORE, OP_SHARED_STORE, OP_LOCAL_STORE):
                addr = [em.pick_reg(), em.pick_reg()] if op == OP_GLOBAL_STORE else [em.pick_reg()]
                data = em.pick_reg()
                rb = U.below(n_bars)
                em.emit(op, g, use_regs=addr + [data], rbar=rb, guard_use=gpred)
                em.pending_store[data] = rb
            elif op == OP_BRANCH:
                # a surplus branch draw: a non-terminating control instruction
                em.emit(op, g, use_preds=[em.pick_pred()], guard_use=gpred)
            elif op == OP_BARRIER:
                if U.u() < 0.5:
                    wb = U.below(n_bars)
                    em.emit(op, g, wbar=wb, guard_use=gpred)
                    em.pending_bar = wb
                else:
                    em.emit(op, g, guard_use=gpred)
            else:  # OP_CALL
                em.emit(op, g, guard_use=gpred)


# ------------------------------------------------------------------ scopes
class _ScopeTree:
    """Scope nodes with a sort key (first global instruction index) used to
    order siblings before preorder numbering."""

    def __init__(self):
        self.parent, self.kind, self.flags, self.key = [], [], [], []

    def add(self, parent, kind, flags=0, key=0):
        self.parent.append(parent)
        self.kind.append(kind)
        self.flags.append(flags)
        self.key.append(key)
        return len(self.parent) - 1

    def preorder(self):
        n = len(self.parent)
        children = [[] for _ in range(n)]
        roots = []
        for s in range(n):
            (roots if self.parent[s] is None else children[self.parent[s]]).append(s)
        for c in children:
            c.sort(key=lambda s: (self.key[s], self.kind[s]))
        roots.sort(key=lambda s: self.key[s])
        order = []
        stack = list(reversed(roots))
        while stack:
            s = stack.pop()
            order.append(s)
            stack.extend(reversed(children[s]))
        remap = np.empty(n, np.int64)
        remap[np.array(order, np.int64)] = np.arange(n)
        return order, remap


def _function_scopes(rng, tree, fscope, block_sizes, loops, base, instr_scope, inline_frac=0.0,
                     math_frac=0.5):
    """Loop scopes mirroring the loop nest and line scopes of 1-8 consecutive
    instructions inside one block; optionally an inlined FUNCTION scope
    (math or device) wrapping a line."""
    nb = len(block_sizes)
    first = np.concatenate([[0], np.cumsum(block_sizes)[:-1]]).astype(np.int64) + base
    loop_scope = {}
    for li in sorted(range(len(loops)), key=lambda i: (loops[i][0], -loops[i][1])):
        h, t = loops[li]
        enclosing = [lj for lj in loop_scope if loops[lj][0] < h and t < loops[lj][1]]
        parent = fscope
        if enclosing:
            parent = loop_scope[min(enclosing, key=lambda lj: loops[lj][1] - loops[lj][0])]
        loop_scope[li] = tree.add(parent, SCOPE_LOOP, 0, int(first[h]))
    for b in range(nb):
        inner = [li for li, (h, t) in enumerate(loops) if h <= b <= t]
        parent = fscope
        if inner:
            parent = loop_scope[min(inner, key=lambda i: loops[i][1] - loops[i][0])]
        k = 0
        size = block_sizes[b]
        while k < size:
            n = int(min(size - k, rng.integers(1, 9)))
            pos = int(first[b]) + k
            line_parent = parent
            if inline_frac > 0 and rng.random() < inline_frac:
                fl = SF_MATH_FN if rng.random() < math_frac else SF_DEVICE_FN
                line_parent = tree.add(parent, SCOPE_FUNCTION, fl, pos)
            sid = tree.add(line_parent, SCOPE_LINE, 0, pos)
            instr_scope[pos - base:pos - base + n] = sid
            k += n


# ---------------------------------------------------------------- programs
def _split_blocks(rng, n_instr, nb, min_size=2):
    extra = n_instr - min_size * nb
    assert extra >= 0, "too few instructions for the block count"
    sizes = min_size + rng.multinomial(extra, np.full(nb, 1.0 / nb))
    return [int(s) for s in sizes]


def gen_program(seed=0, functions=None, n_regs=64, n_preds=8, n_bars=2,
                guard_frac=0.10, pair_frac=0.03, branch_frac=0.25, inline_frac=0.0,
                op_mix=None, rng=None, math_frac=0.5):
    """Generate one program.

    ``functions`` is a list of dicts with keys ``n_instr``, ``n_blocks``,
    ``n_loops``, ``max_depth``, optional ``one_nest_depth``, ``kind``
    ('kernel' | 'device' | 'math'). A 'device'/'math' function becomes a
    FUNCTION scope with its own CFG under the most recent kernel root.
    """
    rng = rng if rng is not None else np.random.default_rng(seed)
    if functions is None:
        functions = [dict(n_instr=2000, n_blocks=40, one_nest_depth=3, kind="kernel")]
    op_mix = op_mix or BASE_OP_MIX
    tree = _ScopeTree()
    all_op, all_guard, all_defs, all_uses = [], [], [], []
    block_begin = [0]
    succ_lists = []
    func_block_begin = [0]
    func_scope_tmp = []
    instr_scope_parts = []
    current_root = None
    for fdesc in functions:
        n = int(fdesc["n_instr"])
        nb = int(fdesc["n_blocks"])
        kind_f = fdesc.get("kind", "kernel")
        sizes = _split_blocks(rng, n, nb)
        loops = _gen_loops(rng, nb, int(fdesc.get("n_loops", 0)), int(fdesc.get("max_depth", 1)),
                           fdesc.get("one_nest_depth"))
        succs, bkind = _build_cfg(rng, nb, loops, branch_frac)
        em = _Emitter(rng, n_regs, n_preds, n_bars)
        _gen_function_body(rng, em, sizes, bkind, op_mix, guard_frac, pair_frac)
        assert len(em.op) == n
        base = len(all_op)
        if kind_f == "kernel" or current_root is None:
            fs = tree.add(None, SCOPE_FUNCTION, SF_KERNEL_ENTRY | SF_HAS_CFG, base)
            current_root = fs
        else:
            fl = SF_HAS_CFG | SF_DEVICE_FN | (SF_MATH_FN if kind_f == "math" else 0)
            fs = tree.add(current_root, SCOPE_FUNCTION, fl, base)
        iscope = np.zeros(n, np.int64)
        _function_scopes(rng, tree, fs, sizes, loops, base, iscope, inline_frac, math_frac)
        instr_scope_parts.append(iscope)
        base_b = len(block_begin) - 1
        for b in range(nb):
            block_begin.append(block_begin[-1] + sizes[b])
            succ_lists.append([base_b + s for s in succs[b]])
        func_block_begin.append(func_block_begin[-1] + nb)
        func_scope_tmp.append(fs)
        all_op += em.op
        all_guard += em.guard
        all_defs += em.defs
        all_uses += em.uses
    order, remap = tree.preorder()
    ns = len(order)
    scope_parent = np.empty(ns, np.uint32)
    scope_kind = np.empty(ns, np.uint8)
    scope_flags = np.empty(ns, np.uint8)
    for new, old in enumerate(order):
        p = tree.parent[old]
        scope_parent[new] = NO_PARENT if p is None else remap[p]
        scope_kind[new] = tree.kind[old]
        scope_flags[new] = tree.flags[old]
    instr_scope = remap[np.concatenate(instr_scope_parts)].astype(np.uint32)
    n_instr = len(all_op)
    def_ptr = np.zeros(n_instr + 1, np.uint32)
    use_ptr = np.zeros(n_instr + 1, np.uint32)
    def_ptr[1:] = np.cumsum([len(d) for d in all_defs])
    use_ptr[1:] = np.cumsum([len(u) for u in all_uses])
    def_loc = np.array([l for d in all_defs for (l, _) in d], np.uint32)
    def_kind = np.array([k for d in all_defs for (_, k) in d], np.uint8)
    use_loc = np.array([l for u in all_uses for (l, _) in u], np.uint32)
    use_kind = np.array([k for u in all_uses for (_, k) in u], np.uint8)
    succ_ptr = np.zeros(len(succ_lists) + 1, np.uint32)
    succ_ptr[1:] = np.cumsum([len(s) for s in succ_lists])
    succ = np.array([s for lst in succ_lists for s in lst], np.uint32)
    arch = default_arch()
    return {
        "n_regs": n_regs, "n_preds": n_preds, "n_bars": n_bars,
        "op_class": np.array(all_op, np.uint8), "guard": np.array(all_guard, np.uint8),
        "def_ptr": def_ptr, "def_loc": def_loc, "def_kind": def_kind,
        "use_ptr": use_ptr, "use_loc": use_loc, "use_kind": use_kind,
        "block_begin": np.array(block_begin, np.uint32),
        "succ_ptr": succ_ptr, "succ": succ,
        "func_block_begin": np.array(func_block_begin, np.uint32),
        "func_scope": remap[np.array(func_scope_tmp, np.int64)].astype(np.uint32),
        "instr_scope": instr_scope,
        "scope_parent": scope_parent, "scope_kind": scope_kind, "scope_flags": scope_flags,
        "lat": arch["lat"], "allowed": arch["allowed"], "blamable": int(arch["blamable"]),
    }


# ----------------------------------------------------------------- samples
def gen_samples(n, n_instr, zipf_s, stall_mix, seed=0, rng=None, pc_base=0,
                latency_frac=0.5, perm=None, out=None):
    """``n`` records with pc ~ Zipf(s) over ranks mapped through a seeded
    permutation of the instructions, stall reason i.i.d. from ``stall_mix``
    and the latency bit ~ Bernoulli(latency_frac) except for SELECTED and
    NOT_SELECTED samples (the scheduler issued)."""
    rng = rng if rng is not None else np.random.default_rng(seed)
    ranks = np.arange(1, n_instr + 1, dtype=np.float64)
    cdf = np.cumsum(ranks ** (-float(zipf_s)))
    cdf /= cdf[-1]
    if perm is None:
        perm = rng.permutation(n_instr).astype(np.uint32)
    rec = np.zeros(n, SAMPLE_DTYPE) if out is None else out
    if out is not None:
        assert len(out) == n and out.dtype == SAMPLE_DTYPE
        rec["reserved"] = 0
    chunk = 1 << 22
    mix_cdf = np.cumsum(np.asarray(stall_mix, np.float64))
    mix_cdf /= mix_cdf[-1]
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        m = e - s
        idx = np.searchsorted(cdf, rng.random(m), side="right")
        np.minimum(idx, n_instr - 1, out=idx)
        rec["pc"][s:e] = perm[idx] + pc_base
        st = np.searchsorted(mix_cdf, rng.random(m), side="right")
        np.minimum(st, N_STALLS - 1, out=st)
        rec["stall"][s:e] = st
        lam = (rng.random(m) < latency_frac) & (st != ST_SELECTED) & (st != ST_NOT_SELECTED)
        rec["flags"][s:e] = lam
    return rec


def corrupt_samples(rec, frac, n_instr, seed=0):
    """Return a copy with ``frac`` of the records made invalid in one of four
    ways (pc out of range, stall out of range, unknown flag bit, nonzero
    reserved field)."""
    rng = np.random.default_rng(seed)
    out = rec.copy()
    k = int(len(out) * frac)
    if k == 0:
        return out
    idx = rng.choice(len(out), size=k, replace=False)
    how = rng.integers(0, 4, size=k)
    out["pc"][idx[how == 0]] = n_instr + rng.integers(0, 1000, size=int((how == 0).sum()))
    out["stall"][idx[how == 1]] = 12 + rng.integers(0, 200, size=int((how == 1).sum()))
    out["flags"][idx[how == 2]] |= (2 << rng.integers(0, 7, size=int((how == 2).sum()))).astype(np.uint8)
    out["reserved"][idx[how == 3]] = 1 + rng.integers(0, 1000, size=int((how == 3).sum()))
    return out


# ---------------------------------------------------------------- workloads
def workload_small(seed=0, n_samples=200_000):
    """2,000 instructions in 40 blocks with one depth-3 loop nest, 64 R + 8 P
    + 2 B; 200k samples with pc Zipf(1.1)."""
    prog = gen_program(seed=seed, functions=[dict(n_instr=2000, n_blocks=40, one_nest_depth=3,
                                                  kind="kernel")],
                       n_regs=64, n_preds=8, n_bars=2)
    rng = np.random.default_rng([seed, 1])
    rec = gen_samples(n_samples, 2000, 1.1, stall_mix_small(), rng=rng)
    return prog, rec


def workload_large(seed=1, n_samples=20_000_000):
    """60,000 instructions in 1,500 blocks, loop depth up to 5, 255 R + 7 P +
    16 B; 20M samples with pc Zipf(1.2), memory dependency 50%."""
    prog = gen_program(seed=seed, functions=[dict(n_instr=60_000, n_blocks=1500, n_loops=100,
                                                  max_depth=5, kind="kernel")],
                       n_regs=255, n_preds=7, n_bars=16)
    rng = np.random.default_rng([seed, 1])
    rec = gen_samples(n_samples, 60_000, 1.2, stall_mix_memory_skewed(), rng=rng)
    return prog, rec


def workload_multi(seed=5, n_kernels=3, n_samples=300_000):
    """A few kernels, each with a device function (own CFG) and inlined
    math/device function scopes; used to cover the multi-function and
    multi-kernel paths at small size."""
    rng = np.random.default_rng(seed)
    funcs = []
    for k in range(n_kernels):
        funcs.append(dict(n_instr=int(rng.integers(300, 900)), n_blocks=int(rng.integers(8, 30)),
                          n_loops=3, max_depth=2, kind="kernel"))
        funcs.append(dict(n_instr=int(rng.integers(60, 200)), n_blocks=int(rng.integers(3, 8)),
                          n_loops=1, max_depth=1, kind="math" if k % 2 else "device"))
    prog = gen_program(functions=funcs, n_regs=32, n_preds=4, n_bars=6, inline_frac=0.08,
                       rng=rng)
    n_instr = len(prog["op_class"])
    # records grouped by kernel: one contiguous segment per kernel's instruction range
    fbb = prog["func_block_begin"]
    bb = prog["block_begin"]
    segs = []
    per = n_samples // n_kernels
    for k in range(n_kernels):
        lo = int(bb[fbb[2 * k]])
        hi = int(bb[fbb[2 * k + 2]])
        segs.append(gen_samples(per, hi - lo, 1.1, stall_mix_small(), rng=rng, pc_base=lo))
    return prog, np.concatenate(segs)


# ------------------------------------------------------- batched workloads
def _lognormal(rng, n, median, sigma, lo, hi):
    return np.clip(np.exp(np.log(median) + sigma * rng.standard_normal(n)), lo, hi)


def _dirichlet_around(rng, mean, concentration_per_category=2.0):
    """A mix drawn from Dirichlet(alpha) with E = mean and total concentration
    `concentration_per_category` times the number of nonzero categories."""
    mean = np.asarray(mean, np.float64)
    nz = mean > 0
    alpha = concentration_per_category * nz.sum() * mean[nz]
    out = np.zeros_like(mean)
    out[nz] = rng.dirichlet(alpha)
    return out


def batch_profile_specs(config: int, seed: int | None = None):
    """Per-profile generation specs of the batched workloads (everything a
    profile's program and records are drawn from; each profile has its own
    seed, so a profile does not depend on how the batch is generated).

    config 2: 1,024 kernel profiles; instructions log-normal (median 3k,
      sigma 1, clipped to 200-60k), records log-normal (median 200k, sigma 1,
      clipped to 10k-10M); opcode and stall mixes Dirichlet around the
      plain-path mixes (concentration 2 per category); Zipf(1.1) PCs.
    config 3: 400 kernels of one application, the same instruction law
      rescaled to 2M instructions in all, and 500M records in all split in
      proportion to log-normal weights (grouped by kernel).
    Both: one FUNCTION scope per about 170 instructions, a tenth of them
    device functions with their own CFG, the rest inlined function scopes
    (2% of all function scopes flagged math)."""
    if config not in (2, 3):
        raise ValueError("batched workloads are configs 2 and 3")
    seed = config if seed is None else seed
    rng = np.random.default_rng([seed, 77])
    if config == 2:
        count = 1024
        n_instr = _lognormal(rng, count, 3000, 1.0, 200, 60_000).astype(np.int64)
        n_rec = _lognormal(rng, count, 200_000, 1.0, 10_000, 10_000_000).astype(np.int64)
    else:
        count = 400
        w = _lognormal(rng, count, 3000, 1.0, 200, 60_000)
        n_instr = np.clip(np.round(w * (2_000_000 / w.sum())), 200, 60_000).astype(np.int64)
        n_instr[-1] += 2_000_000 - int(n_instr.sum())          # exactly 2M in all
        n_instr = np.clip(n_instr, 200, 60_000)
        r = _lognormal(rng, count, 200_000, 1.0, 10_000, 10_000_000)
        n_rec = np.maximum(np.round(r * (500_000_000 / r.sum())), 10_000).astype(np.int64)
        n_rec[-1] += 500_000_000 - int(n_rec.sum())
    stall0 = stall_mix_small()
    op0 = _mix_array(BASE_OP_MIX)
    seeds = np.random.SeedSequence([seed, 2024]).spawn(count)
    specs = []
    for k in range(count):
        op_mix = _dirichlet_around(rng, op0)
        stall_mix = _dirichlet_around(rng, stall0)
        specs.append(dict(index=k, seed=seeds[k], n_instr=int(n_instr[k]), n_rec=int(n_rec[k]),
                          op_mix={c: float(op_mix[c]) for c in range(N_OP_CLASSES) if op_mix[c] > 0},
                          stall_mix=stall_mix, zipf=1.1))
    return specs


def gen_profile_program(spec):
    """The program of one batched profile: a kernel plus device functions
    with their own CFG (a tenth of its function scopes) and inlined function
    scopes, about 45 instructions per block, loops of depth up to 4."""
    rng = np.random.default_rng(spec["seed"])
    n = spec["n_instr"]
    n_fscopes = max(1, round(n / 170))
    n_dev = int(round(0.1 * n_fscopes))
    dev_sizes = []
    rest = n
    for _ in range(n_dev):
        m = int(max(40, min(rest // 4, rng.integers(40, max(41, n // 8)))))
        if rest - m < 100:
            break
        dev_sizes.append(m)
        rest -= m
    funcs = [dict(n_instr=rest, n_blocks=max(2, min(4096, rest // 45)),
                  n_loops=max(1, rest // 45 // 15), max_depth=4, kind="kernel")]
    for m in dev_sizes:
        funcs.append(dict(n_instr=m, n_blocks=max(2, min(4096, m // 45)), n_loops=max(0, m // 45 // 15),
                          max_depth=2, kind="device"))
    n_inl = max(0, n_fscopes - 1 - len(dev_sizes))
    lines = n / 4.5
    inline_frac = min(0.5, n_inl / lines) if lines else 0.0
    regs = 64 if n < 10_000 else (128 if n < 30_000 else 255)
    return gen_program(functions=funcs, n_regs=regs, n_preds=7, n_bars=6, inline_frac=inline_frac,
                       math_frac=0.02, op_mix=spec["op_mix"], rng=rng)


def gen_profile(spec, out=None):
    """One batched profile: (program, records).  `out`, when given, is an
    array of spec['n_rec'] records to fill (and is returned)."""
    prog = gen_profile_program(spec)
    rng = np.random.default_rng([spec["seed"].entropy, 1] + list(spec["seed"].spawn_key))
    rec = gen_samples(spec["n_rec"], len(prog["op_class"]), spec["zipf"], spec["stall_mix"],
                      rng=rng, out=out)
    return prog, rec


def _worker_main(job_file, shm_name, total, out_file):
    """Entry point of one generator worker process (see gen_batch)."""
    import pickle
    from multiprocessing import shared_memory
    with open(job_file, "rb") as f:
        jobs = pickle.load(f)
    shm = shared_memory.SharedMemory(name=shm_name)
    # the creating process owns the segment: this process's resource tracker
    # must not remove it when this process ends
    from multiprocessing import resource_tracker
    resource_tracker.unregister(shm._name, "shared_memory")
    progs = {}
    try:
        view = np.ndarray((total,), SAMPLE_DTYPE, buffer=shm.buf)
        for spec, offset in jobs:
            progs[spec["index"]], _ = gen_profile(spec, out=view[offset:offset + spec["n_rec"]])
        del view
    finally:
        shm.close()
    with open(out_file, "wb") as f:
        pickle.dump(progs, f, protocol=pickle.HIGHEST_PROTOCOL)


def gen_batch(config: int, seed: int | None = None, workers: int | None = None, specs=None):
    """All profiles of a batched workload: (programs, records, offsets);
    profile k's records are records[offsets[k]:offsets[k+1]].  Profiles are
    generated by up to 16 worker processes (fresh Python interpreters started
    as child processes; none when workers <= 1), which write the records
    into shared memory; each profile depends only on its own spec."""
    import os
    import pickle
    import subprocess
    import sys
    import tempfile
    specs = specs if specs is not None else batch_profile_specs(config, seed)
    sizes = np.array([s["n_rec"] for s in specs], np.int64)
    offsets = np.concatenate([[0], np.cumsum(sizes)])
    total = int(offsets[-1])
    if workers is None:
        workers = min(16, os.cpu_count() or 1)
    workers = max(1, min(workers, len(specs)))
    progs = [None] * len(specs)
    if workers <= 1:
        records = np.empty(total, SAMPLE_DTYPE)
        for k, s in enumerate(specs):
            progs[k], _ = gen_profile(s, out=records[offsets[k]:offsets[k + 1]])
        return progs, records, offsets
    from multiprocessing import shared_memory
    # largest first onto the least loaded worker
    cost = [s["n_rec"] + 200 * s["n_instr"] for s in specs]
    groups = [[] for _ in range(workers)]
    load = [0] * workers
    for k in sorted(range(len(specs)), key=lambda k: -cost[k]):
        w = load.index(min(load))
        groups[w].append((specs[k], int(offsets[k])))
        load[w] += cost[k]
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ)
    env["PYTHONPATH"] = root + (os.pathsep + env["PYTHONPATH"] if env.get("PYTHONPATH") else "")
    env["OMP_NUM_THREADS"] = "1"
    shm = shared_memory.SharedMemory(create=True, size=max(8, total * 8))
    try:
        with tempfile.TemporaryDirectory() as td:
            procs = []
            for w, g in enumerate(groups):
                jf, of = os.path.join(td, f"jobs{w}.pkl"), os.path.join(td, f"progs{w}.pkl")
                with open(jf, "wb") as f:
                    pickle.dump(g, f, protocol=pickle.HIGHEST_PROTOCOL)
                code = ("import sys; from paper_2009_04061_amd.synth import _worker_main; "
                        "_worker_main(sys.argv[1], sys.argv[2], int(sys.argv[3]), sys.argv[4])")
                procs.append((subprocess.Popen([sys.executable, "-c", code, jf, shm.name,
                                                str(total), of], cwd=root, env=env), of))
            failed = [p.wait() for p, _ in procs]
            if any(failed):
                raise RuntimeError(f"generator workers failed: exit codes {failed}")
            for _, of in procs:
                with open(of, "rb") as f:
                    for k, prog in pickle.load(f).items():
                        progs[k] = prog
        records = np.empty(total, SAMPLE_DTYPE)
        records[:] = np.ndarray((total,), SAMPLE_DTYPE, buffer=shm.buf)
    finally:
        shm.close()
        shm.unlink()
    return progs, records, offsets


def gen_samples_device(n, n_instr, zipf_s, stall_mix, generator, perm=None,
                       latency_frac=0.5, device="cuda"):
    """Records drawn like gen_samples, but on the GPU with torch (a seeded
    torch.Generator on the device): for the serving workload, whose requests
    are too many to draw on the host.  Returns a uint8 tensor of 8n bytes."""
    import torch
    ranks = torch.arange(1, n_instr + 1, dtype=torch.float64, device=device)
    cdf = torch.cumsum(ranks ** (-float(zipf_s)), 0)
    cdf /= cdf[-1].clone()
    if perm is None:
        perm = torch.randperm(n_instr, generator=generator, device=device)
    mix = torch.as_tensor(np.cumsum(np.asarray(stall_mix, np.float64)), device=device)
    mix /= mix[-1].clone()
    u = torch.rand(n, generator=generator, device=device, dtype=torch.float64)
    idx = torch.clamp(torch.searchsorted(cdf, u, right=True), max=n_instr - 1)
    pc = perm[idx].to(torch.int64)
    u = torch.rand(n, generator=generator, device=device, dtype=torch.float64)
    st = torch.clamp(torch.searchsorted(mix, u, right=True), max=N_STALLS - 1).to(torch.int64)
    u = torch.rand(n, generator=generator, device=device, dtype=torch.float64)
    lam = ((u < latency_frac) & (st != ST_SELECTED) & (st != ST_NOT_SELECTED)).to(torch.int64)
    packed = pc | (st << 32) | (lam << 40)
    return packed.view(torch.uint8)


def serving_specs(seed: int = 4, n_programs: int = 2000):
    """Program specs of the serving workload: resident programs with the
    whole-application instruction law (log-normal, median 3k, sigma 1,
    clipped 200-60k), built like the batched profiles."""
    rng = np.random.default_rng([seed, 88])
    n_instr = _lognormal(rng, n_programs, 3000, 1.0, 200, 60_000).astype(np.int64)
    stall0 = stall_mix_small()
    op0 = _mix_array(BASE_OP_MIX)
    seeds = np.random.SeedSequence([seed, 4242]).spawn(n_programs)
    specs = []
    for k in range(n_programs):
        op_mix = _dirichlet_around(rng, op0)
        stall_mix = _dirichlet_around(rng, stall0)
        specs.append(dict(index=k, seed=seeds[k], n_instr=int(n_instr[k]), n_rec=0,
                          op_mix={c: float(op_mix[c]) for c in range(N_OP_CLASSES) if op_mix[c] > 0},
                          stall_mix=stall_mix, zipf=1.1))
    return specs


def serving_requests(seed: int, n_programs: int, rate: float, seconds: float,
                     lo: int = 50_000, hi: int = 5_000_000):
    """The request stream: Poisson arrivals at `rate` per second over
    `seconds`, a uniformly chosen program and a log-uniform record count in
    [lo, hi] each: (arrival times, program indices, record counts)."""
    rng = np.random.default_rng([seed, 99])
    gaps = rng.exponential(1.0 / rate, size=int(rate * seconds * 1.5) + 16)
    t = np.cumsum(gaps)
    t = t[t < seconds]
    prog = rng.integers(0, n_programs, size=len(t))
    n = np.exp(rng.uniform(np.log(lo), np.log(hi), size=len(t))).astype(np.int64)
    return t, prog, n
