"""A tiny assembler for hand-written test programs in the paper's notation.

Syntax, one item per line (``#`` starts a comment)::

    block 0 -> 1 2          # block 0 with successors 1 and 2, in CSR order
      @P0 LDG R0 <- R2 R3 | wbar B0
      IADD R1 <- R0 R5 | wait B0
    loop 0 1                # a LOOP scope over blocks 0..1 (nested by range)
    func math 3 4           # an inlined FUNCTION scope (math_fn / device_fn) over blocks 3..4
    cfg device              # the blocks that follow form a function with its
                            # own CFG (kernel | device | math); a device or
                            # math function hangs below the latest kernel

Every instruction gets its own LINE scope under the innermost loop (or
function) holding its block.  ``@Pk`` / ``@!Pk`` set the guard and add a
guard use of ``Pk``.  ``Pk`` in the def list defines a predicate.
"""
from __future__ import annotations

import re

import numpy as np

from paper_2009_04061_amd import synth as S

OPS = {
    "MOV": S.OP_ALU, "IADD": S.OP_ALU, "IMAD": S.OP_ALU, "ISETP": S.OP_ALU, "FADD": S.OP_ALU,
    "NOP": S.OP_ALU, "DADD": S.OP_FP64, "DMUL": S.OP_FP64, "F2F": S.OP_LONG_ALU,
    "IDIV": S.OP_LONG_ALU, "LDG": S.OP_GLOBAL_LOAD, "LDS": S.OP_SHARED_LOAD,
    "LDL": S.OP_LOCAL_LOAD, "LDC": S.OP_CONST_LOAD, "STG": S.OP_GLOBAL_STORE,
    "STS": S.OP_SHARED_STORE, "STL": S.OP_LOCAL_STORE, "BRA": S.OP_BRANCH,
    "BAR": S.OP_BARRIER, "CALL": S.OP_CALL,
}


def assemble(text: str, n_regs=16, n_preds=4, n_bars=6, arch=None):
    blocks = []     # list of (succs, [instr dicts])
    loops = []
    funcs = []
    cfgs = [("kernel", 0)]      # (kind, first block) of each function with a CFG
    for raw in text.splitlines():
        line = raw.split("#")[0].strip()
        if not line:
            continue
        if line.startswith("block"):
            m = re.match(r"block\s+(\d+)\s*->\s*(.*)$", line)
            assert m and int(m.group(1)) == len(blocks), line
            succs = [int(t) for t in m.group(2).split()]
            blocks.append((succs, []))
            continue
        if line.startswith("loop"):
            _, a, b = line.split()
            loops.append((int(a), int(b)))
            continue
        if line.startswith("cfg"):
            _, kind = line.split()
            assert kind in ("kernel", "device", "math"), line
            if blocks:
                cfgs.append((kind, len(blocks)))
            else:
                cfgs[0] = (kind, 0)
            continue
        if line.startswith("func"):
            _, kind, a, b = line.split()
            funcs.append((kind, int(a), int(b)))
            continue
        body, _, extra = line.partition("|")
        toks = body.split()
        guard = 0
        gpred = None
        if toks[0].startswith("@"):
            g = toks.pop(0)[1:]
            neg = g.startswith("!")
            gpred = int(g.lstrip("!P"))
            guard = S.guard_literal(gpred, neg)
        op = toks.pop(0)
        defs, uses = [], []
        if "<-" in toks:
            k = toks.index("<-")
            dtok, utok = toks[:k], toks[k + 1:]
        else:
            dtok, utok = toks, []
        for t in dtok:
            if t.startswith("R"):
                defs.append((int(t[1:]), S.DEF_REG))
            elif t.startswith("P"):
                defs.append((n_regs + int(t[1:]), S.DEF_PRED))
        if gpred is not None:
            uses.append((n_regs + gpred, S.USE_GUARD))
        for t in utok:
            if t.startswith("R"):
                uses.append((int(t[1:]), S.USE_OPND))
            elif t.startswith("P"):
                uses.append((n_regs + int(t[1:]), S.USE_OPND))
        for clause in extra.split(","):
            clause = clause.strip()
            if not clause:
                continue
            key, val = clause.split()
            for v in val.split("+"):
                loc = n_regs + n_preds + int(v.strip()[1:])
                if key == "wbar":
                    defs.append((loc, S.DEF_WBAR))
                elif key == "rbar":
                    defs.append((loc, S.DEF_RBAR))
                elif key == "wait":
                    uses.append((loc, S.USE_WAIT))
                else:
                    raise ValueError(clause)
        blocks[-1][1].append(dict(op=OPS[op], guard=guard, defs=defs, uses=uses))
    nb = len(blocks)
    ins = [i for _, lst in blocks for i in lst]
    n = len(ins)
    block_begin = np.zeros(nb + 1, np.uint32)
    block_begin[1:] = np.cumsum([len(lst) for _, lst in blocks])
    # scopes: one FUNCTION per CFG function (a kernel is a root, a device or
    # math function hangs below the latest kernel), loops and inlined
    # functions nested by block range inside their CFG function, one line
    # per instruction
    nf = len(cfgs)
    fbb = [b0 for _, b0 in cfgs] + [nb]
    func_of = np.zeros(nb, np.int64)
    for f in range(nf):
        func_of[fbb[f]:fbb[f + 1]] = f
    parent, kind, flags, key = [], [], [], []
    fscope = []
    last_kernel = None
    for f, (k, b0) in enumerate(cfgs):
        fl = S.SF_HAS_CFG
        if k == "kernel":
            fl |= S.SF_KERNEL_ENTRY
            par = None
        else:
            fl |= S.SF_DEVICE_FN | (S.SF_MATH_FN if k == "math" else 0)
            assert last_kernel is not None, "a device function needs a kernel before it"
            par = last_kernel
        parent.append(par)
        kind.append(S.SCOPE_FUNCTION)
        flags.append(fl)
        key.append(int(block_begin[b0]))
        fscope.append(len(parent) - 1)
        if k == "kernel":
            last_kernel = len(parent) - 1
    regions = [("loop", a, b) for a, b in loops] + [(k, a, b) for k, a, b in funcs]
    regions.sort(key=lambda r: (r[1], -r[2]))
    for (_, a, b) in regions:
        assert func_of[a] == func_of[b], "a region must stay inside one function"
    reg_scope = []
    for (k, a, b) in regions:
        enclosing = [ri for ri, (_, a2, b2) in enumerate(regions[:len(reg_scope)])
                     if a2 <= a and b <= b2]
        par = (fscope[func_of[a]] if not enclosing
               else reg_scope[max(enclosing, key=lambda ri: regions[ri][1])])
        parent.append(par)
        if k == "loop":
            kind.append(S.SCOPE_LOOP)
            flags.append(0)
        else:
            kind.append(S.SCOPE_FUNCTION)
            flags.append(S.SF_MATH_FN if k == "math" else S.SF_DEVICE_FN)
        key.append(int(block_begin[a]))
        reg_scope.append(len(parent) - 1)
    instr_scope_tmp = []
    for b in range(nb):
        inner = [ri for ri, (_, a, e) in enumerate(regions) if a <= b <= e]
        par = (fscope[func_of[b]] if not inner
               else reg_scope[min(inner, key=lambda ri: (regions[ri][2] - regions[ri][1], -ri))])
        for t in range(int(block_begin[b]), int(block_begin[b + 1])):
            parent.append(par)
            kind.append(S.SCOPE_LINE)
            flags.append(0)
            key.append(t)
            instr_scope_tmp.append(len(parent) - 1)
    ns = len(parent)
    children = [[] for _ in range(ns)]
    roots = []
    for s in range(ns):
        (roots if parent[s] is None else children[parent[s]]).append(s)
    for c in children:
        c.sort(key=lambda s: (key[s], kind[s]))
    roots.sort(key=lambda s: key[s])
    order, stack = [], list(reversed(roots))
    while stack:
        s = stack.pop()
        order.append(s)
        stack.extend(reversed(children[s]))
    remap = np.empty(ns, np.int64)
    remap[np.array(order)] = np.arange(ns)
    scope_parent = np.array([S.NO_PARENT if parent[o] is None else remap[parent[o]] for o in order],
                            np.uint32)
    arch = arch or S.default_arch()
    def_ptr = np.zeros(n + 1, np.uint32)
    def_ptr[1:] = np.cumsum([len(i["defs"]) for i in ins])
    use_ptr = np.zeros(n + 1, np.uint32)
    use_ptr[1:] = np.cumsum([len(i["uses"]) for i in ins])
    succ_ptr = np.zeros(nb + 1, np.uint32)
    succ_ptr[1:] = np.cumsum([len(s) for s, _ in blocks])
    return {
        "n_regs": n_regs, "n_preds": n_preds, "n_bars": n_bars,
        "op_class": np.array([i["op"] for i in ins], np.uint8),
        "guard": np.array([i["guard"] for i in ins], np.uint8),
        "def_ptr": def_ptr,
        "def_loc": np.array([l for i in ins for l, _ in i["defs"]], np.uint32),
        "def_kind": np.array([k for i in ins for _, k in i["defs"]], np.uint8),
        "use_ptr": use_ptr,
        "use_loc": np.array([l for i in ins for l, _ in i["uses"]], np.uint32),
        "use_kind": np.array([k for i in ins for _, k in i["uses"]], np.uint8),
        "block_begin": block_begin, "succ_ptr": succ_ptr,
        "succ": np.array([t for s, _ in blocks for t in s], np.uint32),
        "func_block_begin": np.array(fbb, np.uint32),
        "func_scope": remap[np.array(fscope, np.int64)].astype(np.uint32),
        "instr_scope": remap[np.array(instr_scope_tmp, np.int64)].astype(np.uint32),
        "scope_parent": scope_parent,
        "scope_kind": np.array([kind[o] for o in order], np.uint8),
        "scope_flags": np.array([flags[o] for o in order], np.uint8),
        "lat": arch["lat"], "allowed": arch["allowed"], "blamable": int(arch["blamable"]),
    }


def samples(spec) -> np.ndarray:
    """``spec``: iterable of (pc, stall, latency_bit, count)."""
    rows = []
    for pc, stall, lam, cnt in spec:
        rows += [(pc, stall, lam, 0)] * cnt
    rec = np.zeros(len(rows), S.SAMPLE_DTYPE)
    if rows:
        a = np.array(rows)
        rec["pc"], rec["stall"], rec["flags"], rec["reserved"] = a[:, 0], a[:, 1], a[:, 2], a[:, 3]
    return rec


def use_index(prog, instr, loc, kind=None):
    """Index in the use CSR of instruction ``instr``'s use of ``loc``."""
    for u in range(int(prog["use_ptr"][instr]), int(prog["use_ptr"][instr + 1])):
        if int(prog["use_loc"][u]) == loc and (kind is None or int(prog["use_kind"][u]) == kind):
            return u
    raise KeyError((instr, loc))
