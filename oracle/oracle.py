"""Python face of the CPU oracle (TEST INFRASTRUCTURE ONLY).

Loads ``liboracle.so`` (plain C, built from ``gpa_oracle.c`` with gcc) and
marshals numpy arrays.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark use this module; the HIP library never does.
"""
from __future__ import annotations

import contextlib
import ctypes as ct
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
N_OPT = 9
N_FINE = 8
NONE = 0xFFFFFFFF


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, single thread, no intrinsics)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-shared", "-fPIC",
                               "-o", tmp, os.path.join(HERE, "gpa_oracle.c"), "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


def build_variant(source: str, out_path: str) -> str:
    """Compile C source text (a modified copy of the oracle, for the tests
    that plant mistakes in it) into out_path with the same flags."""
    src = out_path + ".c"
    with open(src, "w") as f:
        f.write(source)
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-w", "-shared", "-fPIC", "-I", HERE,
                           "-o", out_path, src, "-lm"])
    return out_path


@contextlib.contextmanager
def use_library(path: str):
    """Route every oracle call to another build of the oracle for a while."""
    global _lib
    saved = _lib
    _lib = _load(path)
    try:
        yield
    finally:
        _lib = saved


class _Prog(ct.Structure):
    _fields_ = [("n_instr", ct.c_uint32), ("n_blocks", ct.c_uint32), ("n_funcs", ct.c_uint32),
                ("n_scopes", ct.c_uint32), ("n_regs", ct.c_uint32), ("n_preds", ct.c_uint32),
                ("n_bars", ct.c_uint32),
                ("op_class", ct.c_void_p), ("guard", ct.c_void_p),
                ("def_ptr", ct.c_void_p), ("def_loc", ct.c_void_p), ("def_kind", ct.c_void_p),
                ("use_ptr", ct.c_void_p), ("use_loc", ct.c_void_p), ("use_kind", ct.c_void_p),
                ("block_begin", ct.c_void_p), ("succ_ptr", ct.c_void_p), ("succ", ct.c_void_p),
                ("func_block_begin", ct.c_void_p), ("func_scope", ct.c_void_p),
                ("instr_scope", ct.c_void_p), ("scope_parent", ct.c_void_p),
                ("scope_kind", ct.c_void_p), ("scope_flags", ct.c_void_p),
                ("lat", ct.c_void_p), ("allowed", ct.c_void_p), ("blamable", ct.c_uint32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build(force=False)
        _lib = _load(LIB_PATH)
    return _lib


def _load(path):
    L = ct.CDLL(path)
    vp, u32, u64 = ct.c_void_p, ct.c_uint32, ct.c_uint64
    L.orc_count.argtypes = [u32, vp, u64, vp, vp]
    L.orc_ctx_new.argtypes = [ct.POINTER(_Prog)]
    L.orc_ctx_new.restype = vp
    L.orc_ctx_free.argtypes = [vp]
    L.orc_sources.argtypes = [vp, u32, ct.c_int, vp, u32]
    L.orc_sources.restype = u32
    L.orc_dist.argtypes = [vp, u32, u32, vp, vp]
    L.orc_dist.restype = ct.c_int
    L.orc_analyze.argtypes = [vp]
    L.orc_analyze.restype = vp
    L.orc_analysis_free.argtypes = [vp]
    L.orc_analysis_sizes.argtypes = [vp, vp, vp]
    L.orc_analysis_rd.argtypes = [vp, vp, vp, vp]
    L.orc_analysis_edges.argtypes = [vp, vp, vp, vp, vp, vp]
    L.orc_blame.argtypes = [vp, vp, vp, vp, vp, vp]
    L.orc_estimate.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, u32, vp, vp, vp]
    L.orc_parallel.argtypes = [vp, vp, u32, vp, vp, vp]
    L.orc_coverage.argtypes = [vp, vp, vp]
    L.orc_hotspots.argtypes = [vp, vp, vp, vp, u32, u32, u32, vp]
    L.orc_hotspots.restype = u32
    return L


def _p(a):
    return a.ctypes.data_as(ct.c_void_p)


def count(n_instr: int, records: np.ndarray):
    """Per-instruction x stall-reason x latency-bit counts and dropped count."""
    raw = np.ascontiguousarray(records).view(np.uint8)
    n = raw.size // 8
    C = np.zeros(n_instr * 24, np.uint32)
    dropped = np.zeros(1, np.uint64)
    lib().orc_count(n_instr, _p(raw), n, _p(C), _p(dropped))
    return C.reshape(n_instr, 12, 2), int(dropped[0])


_FIELDS = [("op_class", np.uint8), ("guard", np.uint8), ("def_ptr", np.uint32),
           ("def_loc", np.uint32), ("def_kind", np.uint8), ("use_ptr", np.uint32),
           ("use_loc", np.uint32), ("use_kind", np.uint8), ("block_begin", np.uint32),
           ("succ_ptr", np.uint32), ("succ", np.uint32), ("func_block_begin", np.uint32),
           ("func_scope", np.uint32), ("instr_scope", np.uint32), ("scope_parent", np.uint32),
           ("scope_kind", np.uint8), ("scope_flags", np.uint8), ("lat", np.uint16),
           ("allowed", np.uint16)]


class Program:
    """A program held by the oracle; keeps the numpy arrays alive."""

    def __init__(self, prog: dict):
        self.arrays = {k: np.ascontiguousarray(np.asarray(prog[k]), dtype=t) for k, t in _FIELDS}
        a = self.arrays
        self.n_instr = len(a["op_class"])
        self.n_scopes = len(a["scope_parent"])
        self.n_uses = int(a["use_ptr"][-1])
        self.blamable = int(prog["blamable"])
        self.n_blamable = bin(self.blamable & 0xFFF).count("1")
        s = _Prog()
        s.n_instr = self.n_instr
        s.n_blocks = len(a["block_begin"]) - 1
        s.n_funcs = len(a["func_block_begin"]) - 1
        s.n_scopes = self.n_scopes
        s.n_regs, s.n_preds, s.n_bars = int(prog["n_regs"]), int(prog["n_preds"]), int(prog["n_bars"])
        for k, _ in _FIELDS:
            setattr(s, k, a[k].ctypes.data)
        s.blamable = self.blamable
        self._s = s
        self.ctx = lib().orc_ctx_new(ct.byref(s))
        self._an = None

    def __del__(self):
        try:
            if self._an:
                lib().orc_analysis_free(self._an)
            if self.ctx:
                lib().orc_ctx_free(self.ctx)
        except Exception:
            pass

    # ------------------------------------------------------------ per item
    def sources(self, use_idx: int, blocked: bool = False) -> np.ndarray:
        cap = 4096
        while True:
            out = np.zeros(cap, np.uint32)
            n = lib().orc_sources(self.ctx, int(use_idx), int(bool(blocked)), _p(out), cap)
            if n <= cap:
                return out[:n].copy()
            cap = int(n)

    def dist(self, i: int, j: int):
        a = np.zeros(1, np.uint32)
        b = np.zeros(1, np.uint32)
        ok = lib().orc_dist(self.ctx, int(i), int(j), _p(a), _p(b))
        return (int(a[0]), int(b[0])) if ok else None

    # -------------------------------------------------------------- whole
    def analyze(self) -> dict:
        L = lib()
        if self._an is None:
            self._an = L.orc_analyze(self.ctx)
        n_rd = np.zeros(1, np.uint64)
        n_e = np.zeros(1, np.uint64)
        L.orc_analysis_sizes(self._an, _p(n_rd), _p(n_e))
        nrd, ne = int(n_rd[0]), int(n_e[0])
        rd_ptr = np.zeros(self.n_uses + 1, np.uint32)
        rd_src = np.zeros(max(nrd, 1), np.uint32)
        rd_blk = np.zeros(max(nrd, 1), np.uint8)
        L.orc_analysis_rd(self._an, _p(rd_ptr), _p(rd_src), _p(rd_blk))
        src = np.zeros(max(ne, 1), np.uint32)
        dst = np.zeros(max(ne, 1), np.uint32)
        flags = np.zeros(max(ne, 1), np.uint8)
        dmin = np.zeros(max(ne, 1), np.uint32)
        dmax = np.zeros(max(ne, 1), np.uint32)
        L.orc_analysis_edges(self._an, _p(src), _p(dst), _p(flags), _p(dmin), _p(dmax))
        return {"rd_ptr": rd_ptr, "rd_src": rd_src[:nrd], "rd_blocked": rd_blk[:nrd],
                "src": src[:ne], "dst": dst[:ne], "flags": flags[:ne], "dmin": dmin[:ne],
                "dmax": dmax[:ne], "n_edges": ne}

    def blame(self, C: np.ndarray) -> dict:
        if self._an is None:
            self.analyze()
        C = np.ascontiguousarray(C, np.uint32).reshape(-1)
        ne = np.zeros(1, np.uint64)
        nrd = np.zeros(1, np.uint64)
        lib().orc_analysis_sizes(self._an, _p(nrd), _p(ne))
        ne = int(ne[0])
        nb = self.n_blamable
        share = np.zeros(max(ne * nb * 2, 1), np.float64)
        blamed = np.zeros(self.n_instr * 24, np.float64)
        self_ = np.zeros(self.n_instr * 24, np.float64)
        fine = np.zeros(self.n_instr * N_FINE * 2, np.float64)
        lib().orc_blame(self._an, _p(C), _p(share), _p(blamed), _p(self_), _p(fine))
        return {"share": share[:ne * nb * 2].reshape(ne, nb, 2),
                "blamed": blamed.reshape(-1, 12, 2), "self": self_.reshape(-1, 12, 2),
                "fine": fine.reshape(-1, N_FINE, 2)}

    def estimate(self, C: np.ndarray, bl: dict, k: int = 5) -> dict:
        C = np.ascontiguousarray(C, np.uint32).reshape(-1)
        ns = self.n_scopes
        share = np.ascontiguousarray(bl["share"], np.float64).reshape(-1)
        if share.size == 0:
            share = np.zeros(1)
        blamed = np.ascontiguousarray(bl["blamed"], np.float64).reshape(-1)
        self_ = np.ascontiguousarray(bl["self"], np.float64).reshape(-1)
        active = np.zeros(ns)
        matched = np.zeros(ns * N_OPT)
        speed = np.zeros(ns * N_OPT)
        root_of = np.zeros(ns, np.uint32)
        kT = np.zeros(ns)
        kL = np.zeros(ns)
        eq3 = np.zeros(ns * 3)
        topo = np.zeros(ns * k, np.uint32)
        tops = np.zeros(ns * k, np.uint32)
        topv = np.zeros(ns * k)
        lib().orc_estimate(self._an, _p(C), _p(share), _p(blamed), _p(self_), _p(active),
                           _p(matched), _p(speed), _p(root_of), _p(kT), _p(kL), _p(eq3), k,
                           _p(topo), _p(tops), _p(topv))
        return {"active": active, "matched": matched.reshape(ns, N_OPT),
                "speedup": speed.reshape(ns, N_OPT), "root_of": root_of, "kernel_T": kT,
                "kernel_L": kL, "eq3": eq3.reshape(ns, 3), "top_opt": topo.reshape(ns, k),
                "top_scope": tops.reshape(ns, k), "top_speed": topv.reshape(ns, k)}


PARALLEL_FIELDS = ["matched", "W", "W_new", "R_I", "I", "I_new", "C_W", "C_I", "f", "speedup"]
LAUNCH_FIELDS = ["blocks", "threads_per_block", "regs_per_thread", "shared_per_block"]
DEVICE_FIELDS = ["n_sm", "schedulers_per_sm", "warp_size", "max_warps_per_sm",
                 "max_blocks_per_sm", "max_threads_per_block", "regs_per_sm", "shared_per_sm"]


def parallel(P: "Program", C: np.ndarray, root: int, launch: dict, device: dict):
    """Block Increase and Thread Increase (Sec. 5.2, Eqs. (6)-(10)) for the
    kernel root scope `root`: two dicts of PARALLEL_FIELDS."""
    if P._an is None:
        P.analyze()
    C = np.ascontiguousarray(C, np.uint32).reshape(-1)
    la = np.array([launch[f] for f in LAUNCH_FIELDS], np.uint32)
    de = np.array([device[f] for f in DEVICE_FIELDS], np.uint32)
    out = np.zeros(22)
    lib().orc_parallel(P._an, _p(C), int(root), _p(la), _p(de), _p(out))
    return [{f: float(out[11 * o + k]) for k, f in enumerate(PARALLEL_FIELDS)} for o in (0, 1)]


def coverage(P: "Program"):
    """Single dependency coverage counts (before, after pruning)."""
    if P._an is None:
        P.analyze()
    b = np.zeros(1, np.uint64)
    a = np.zeros(1, np.uint64)
    lib().orc_coverage(P._an, _p(b), _p(a))
    return int(b[0]), int(a[0])


def hotspots(P: "Program", C, bl: dict, root: int, opt: int, k: int = 5):
    """Hotspots of optimizer `opt` in the kernel rooted at scope `root`:
    list of (src, dst, dmin, dmax, samples)."""
    if P._an is None:
        P.analyze()
    C = np.ascontiguousarray(C, np.uint32).reshape(-1)
    share = np.ascontiguousarray(bl["share"], np.float64).reshape(-1)
    if share.size == 0:
        share = np.zeros(1)
    self_ = np.ascontiguousarray(bl["self"], np.float64).reshape(-1)
    out = np.zeros(5 * max(k, 1))
    n = lib().orc_hotspots(P._an, _p(C), _p(share), _p(self_), int(root), int(opt), int(k), _p(out))
    rows = out[:5 * n].reshape(n, 5)
    return [(int(r[0]), int(r[1]), int(r[2]), int(r[3]), float(r[4])) for r in rows]


def run_all(prog: dict, records: np.ndarray, k: int = 5) -> dict:
    """Counts, analysis, blame and estimates for one program and profile."""
    P = Program(prog)
    C, dropped = count(P.n_instr, records)
    an = P.analyze()
    bl = P.blame(C)
    est = P.estimate(C, bl, k)
    return {"C": C, "dropped": dropped, "analysis": an, "blame": bl, "estimate": est,
            "program": P}
