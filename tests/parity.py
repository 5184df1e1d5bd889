"""GPU-vs-oracle comparison used by the GPU tests and the smoke check.

Tolerances (derived from the arithmetic):
  * counts, totals, per-use source lists, edges, flags, dmin, dmax: bit-exact;
  * FP64 shares, blamed / kept / fine tables: relative 1e-12 (both sides form
    the same products and sum the same terms in the same edge order);
  * matched and active samples per scope: relative 1e-10 (sums of up to ~1e5
    positive terms in a different order: error <= n * 2^-52 relative);
  * speedups: absolute-relative 1e-9; top-k: same speedups rank by rank, and
    the same (optimizer, scope) unless the speedups tie within 1e-9.
"""
from __future__ import annotations

import numpy as np

RTOL_FP = 1e-12
RTOL_SUM = 1e-10
TOL_SPEEDUP = 1e-9
N_STALLS, N_OP_CLASSES = 12, 13


def run_gpu(prog: dict, rec: np.ndarray, device_inputs: bool = True, k: int = 5):
    import torch
    from paper_2009_04061_amd import gpa
    if device_inputs:
        P = gpa.Program(gpa.program_to_device(prog))
        raw = np.ascontiguousarray(rec).view(np.uint8)
        samples = torch.from_numpy(raw.copy()).cuda() if raw.size else torch.zeros(0, dtype=torch.uint8, device="cuda")
    else:
        P = gpa.Program(prog)
        samples = np.ascontiguousarray(rec)
    B = P.attribute(samples)
    A = B.advise()
    C, tot = B.counts()
    out = {"C": C, "totals": tot, "rd": P.rd(), "edges": P.edges(), "shares": B.shares(),
           "table": B.table(), "est": A.get(), "top": A.topk(k), "roots": P.roots(), "info": P.info}
    A.close()
    B.close()
    P.close()
    return out


def with_blamable(prog, mask, seed):
    """The program with another architecture's blamable set: each reason
    newly blamable allows a random set of opcode classes (one allows none,
    so its samples find no candidate)."""
    p = dict(prog)
    al = np.array(prog["allowed"], np.uint16).copy()
    rng = np.random.default_rng([seed, mask])
    fresh = [r for r in range(N_STALLS) if (mask >> r) & 1 and not (prog["blamable"] >> r) & 1]
    for i, r in enumerate(fresh):
        al[r] = 0 if i == 0 else int(rng.integers(1, 1 << N_OP_CLASSES))
    p["allowed"] = al
    p["blamable"] = mask
    return p


def _close(a, b, rtol, what):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    assert a.shape == b.shape, (what, a.shape, b.shape)
    bad = ~(np.abs(a - b) <= rtol * np.maximum(np.abs(a), np.abs(b)))
    bad &= ~((a == b) | (np.isinf(a) & np.isinf(b) & (np.sign(a) == np.sign(b))))
    if bad.any():
        idx = np.argwhere(bad)[:5]
        raise AssertionError(f"{what}: {int(bad.sum())} mismatches, first {idx.tolist()} "
                             f"gpu={a[tuple(idx[0])]!r} oracle={b[tuple(idx[0])]!r}")


def _equal(a, b, what):
    a = np.asarray(a)
    b = np.asarray(b)
    assert a.shape == b.shape, (what, a.shape, b.shape)
    if not np.array_equal(a, b):
        idx = np.nonzero(a.reshape(-1) != b.reshape(-1))[0][:5]
        raise AssertionError(f"{what}: {int((a != b).sum())} mismatches at {idx.tolist()} "
                             f"gpu={a.reshape(-1)[idx].tolist()} oracle={b.reshape(-1)[idx].tolist()}")


def compare(prog: dict, g: dict, o: dict, k: int = 5):
    """Assert the GPU result `g` equals the oracle result `o` (oracle.run_all)."""
    C = o["C"]
    _equal(g["C"], C, "counts")
    _equal(int(g["totals"][0]), int(C.sum()), "valid samples")
    _equal(int(g["totals"][1]), int(C[:, :, 1].sum()), "latency samples")
    _equal(int(g["totals"][2]), int(o["dropped"]), "dropped records")
    an = o["analysis"]
    _equal(g["rd"]["rd_ptr"], an["rd_ptr"], "rd_ptr")
    _equal(g["rd"]["rd_src"], an["rd_src"], "rd_src")
    _equal(g["rd"]["rd_blocked"], an["rd_blocked"], "rd_blocked")
    e = g["edges"]
    for key in ("src", "dst", "flags", "dmin", "dmax"):
        _equal(e[key], an[key], "edge " + key)
    bl = o["blame"]
    _close(g["shares"], bl["share"], RTOL_FP, "shares")
    _close(g["table"]["blamed"], bl["blamed"], RTOL_FP, "blamed")
    _close(g["table"]["self"], bl["self"], RTOL_FP, "kept")
    _close(g["table"]["fine"], bl["fine"], RTOL_FP, "fine")
    est, oe = g["est"], o["estimate"]
    _close(est["active"], oe["active"], RTOL_SUM, "active")
    _close(est["matched"], oe["matched"], RTOL_SUM, "matched")
    _close(est["speedup"], oe["speedup"], TOL_SPEEDUP, "speedup")
    _close(est["kernel_T"], oe["kernel_T"] * (prog["scope_parent"] == 0xFFFFFFFF), RTOL_SUM, "T")
    _close(est["kernel_L"], oe["kernel_L"] * (prog["scope_parent"] == 0xFFFFFFFF), RTOL_SUM, "L")
    roots = np.nonzero(np.asarray(prog["scope_parent"]) == 0xFFFFFFFF)[0]
    _close(est["eq3"][roots], oe["eq3"][roots], TOL_SPEEDUP, "eq3")
    top = g["top"]
    osp = oe["speedup"]
    assert np.array_equal(g["roots"], roots), "kernel roots"
    gsp = np.asarray(est["speedup"])
    for ri, r in enumerate(roots):
        _close(top["top_speed"][ri], oe["top_speed"][r][:k], TOL_SPEEDUP, f"top-k speed root {r}")
        # the GPU's own row: distinct items, each carrying its own speedup,
        # in non-increasing order (whatever the oracle's tie order)
        real = [(int(top["top_opt"][ri, t]), int(top["top_scope"][ri, t]), float(top["top_speed"][ri, t]))
                for t in range(k) if int(top["top_opt"][ri, t]) != 0xFFFFFFFF]
        assert len({(o, l) for o, l, _ in real}) == len(real), ("top-k repeats an item", r)
        for o, l, v in real:
            assert v == gsp[l, o], ("top-k speed is not the item's", r, o, l)
        assert all(a[2] >= b[2] for a, b in zip(real, real[1:])), ("top-k order", r)
        for t in range(k):
            go, gs = int(top["top_opt"][ri, t]), int(top["top_scope"][ri, t])
            oo, os_ = int(oe["top_opt"][r, t]), int(oe["top_scope"][r, t])
            if (go, gs) == (oo, os_):
                continue
            assert go != 0xFFFFFFFF and oo != 0xFFFFFFFF, ("top-k length", r, t)
            v_g, v_o = osp[gs, go], osp[os_, oo]
            assert abs(v_g - v_o) <= TOL_SPEEDUP * max(1.0, abs(v_o)), ("top-k", r, t, go, gs, oo, os_)
