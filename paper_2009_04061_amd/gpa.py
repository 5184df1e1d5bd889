"""ctypes binding of libgpa (include/gpa.h): argument marshalling only.

Every step of the analysis runs in the library's HIP kernels; this module
moves arrays into the descriptor structs, passes device pointers of torch
tensors (or host pointers of numpy arrays) and copies results out.  There is
no fallback: if the compiled library is missing, importing fails.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgpa.so")

N_OPT = 9
N_FINE = 8
NONE = 0xFFFFFFFF

GPA_OK = 0
STATUS = {0: "GPA_OK", -1: "GPA_E_INVALID", -2: "GPA_E_NOMEM", -3: "GPA_E_DEVICE",
          -4: "GPA_E_STATE", -6: "GPA_E_UNSUPPORTED"}


class GpaError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Arch(ct.Structure):
    _fields_ = [("lat", ct.c_uint16 * 16), ("allowed", ct.c_uint16 * 12),
                ("blamable", ct.c_uint16), ("pad", ct.c_uint16)]


class ProgramDesc(ct.Structure):
    _fields_ = [("n_instr", ct.c_uint32), ("n_blocks", ct.c_uint32), ("n_funcs", ct.c_uint32),
                ("n_scopes", ct.c_uint32), ("n_regs", ct.c_uint32), ("n_preds", ct.c_uint32),
                ("n_bars", ct.c_uint32), ("on_device", ct.c_int32),
                ("op_class", ct.c_void_p), ("guard", ct.c_void_p), ("def_ptr", ct.c_void_p),
                ("def_loc", ct.c_void_p), ("def_kind", ct.c_void_p), ("use_ptr", ct.c_void_p),
                ("use_loc", ct.c_void_p), ("use_kind", ct.c_void_p),
                ("block_begin", ct.c_void_p), ("succ_ptr", ct.c_void_p), ("succ", ct.c_void_p),
                ("func_block_begin", ct.c_void_p), ("func_scope", ct.c_void_p),
                ("instr_scope", ct.c_void_p), ("scope_parent", ct.c_void_p),
                ("scope_kind", ct.c_void_p), ("scope_flags", ct.c_void_p), ("arch", Arch)]


class ProgramInfo(ct.Structure):
    _fields_ = [("n_instr", ct.c_uint64), ("n_blocks", ct.c_uint64), ("n_funcs", ct.c_uint64),
                ("n_scopes", ct.c_uint64), ("n_defs", ct.c_uint64), ("n_uses", ct.c_uint64),
                ("n_rd", ct.c_uint64), ("n_edges", ct.c_uint64), ("n_blamable", ct.c_uint32),
                ("n_roots", ct.c_uint32)]


# every entry point declared in include/gpa.h
EXPORTS = ["gpa_load_program", "gpa_program_free", "gpa_program_get_info", "gpa_program_roots",
           "gpa_program_rd",
           "gpa_program_edges", "gpa_attribute", "gpa_blame_free", "gpa_blame_counts",
           "gpa_blame_shares", "gpa_blame_table", "gpa_advise", "gpa_advice_free",
           "gpa_advice_get", "gpa_advice_topk", "gpa_last_error", "gpa_timing_enable",
           "gpa_timing_read"]
PHASES = ["hist", "blame", "load", "advise", "rd_edges", "dist", "dfs", "rd_search",
          "validate", "sites", "edges", "targets", "dist_long"]

_lib = None


def lib():
    """Load libgpa.so (built by paper_2009_04061_amd/build.py)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run paper_2009_04061_amd/build.py "
                              "(there is no fallback path)")
        L = ct.CDLL(LIB_PATH)
        vp, u32, u64, i32 = ct.c_void_p, ct.c_uint32, ct.c_uint64, ct.c_int
        pp = ct.POINTER(ct.c_void_p)
        L.gpa_load_program.argtypes = [ct.POINTER(ProgramDesc), vp, pp]
        L.gpa_program_free.argtypes = [vp]
        L.gpa_program_free.restype = None
        L.gpa_program_get_info.argtypes = [vp, ct.POINTER(ProgramInfo)]
        L.gpa_program_roots.argtypes = [vp, vp]
        L.gpa_program_rd.argtypes = [vp, vp, vp, vp]
        L.gpa_program_edges.argtypes = [vp, vp, vp, vp, vp, vp]
        L.gpa_attribute.argtypes = [vp, vp, u64, i32, vp, pp]
        L.gpa_blame_free.argtypes = [vp]
        L.gpa_blame_free.restype = None
        L.gpa_blame_counts.argtypes = [vp, vp, vp]
        L.gpa_blame_shares.argtypes = [vp, vp]
        L.gpa_blame_table.argtypes = [vp, vp, vp, vp]
        L.gpa_advise.argtypes = [vp, vp, pp]
        L.gpa_advice_free.argtypes = [vp]
        L.gpa_advice_free.restype = None
        L.gpa_advice_get.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        L.gpa_advice_topk.argtypes = [vp, u32, vp, vp, vp]
        L.gpa_timing_enable.argtypes = [i32]
        L.gpa_timing_enable.restype = None
        L.gpa_timing_read.argtypes = [vp, vp, u32, i32]
        L.gpa_timing_read.restype = u32
        L.gpa_last_error.argtypes = []
        L.gpa_last_error.restype = ct.c_char_p
        for name in ("gpa_load_program", "gpa_program_get_info", "gpa_program_rd",
                     "gpa_program_edges", "gpa_attribute", "gpa_blame_counts",
                     "gpa_blame_shares", "gpa_blame_table", "gpa_advise", "gpa_advice_get",
                     "gpa_advice_topk"):
            getattr(L, name).restype = ct.c_int32
        _lib = L
    return _lib


def _check(st):
    if st != GPA_OK:
        raise GpaError(st, lib().gpa_last_error().decode(errors="replace"))


def _ptr(a):
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()   # torch tensor


def _stream(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream or None
    return stream.cuda_stream or None


_DESC_FIELDS = [("op_class", np.uint8), ("guard", np.uint8), ("def_ptr", np.uint32),
                ("def_loc", np.uint32), ("def_kind", np.uint8), ("use_ptr", np.uint32),
                ("use_loc", np.uint32), ("use_kind", np.uint8), ("block_begin", np.uint32),
                ("succ_ptr", np.uint32), ("succ", np.uint32), ("func_block_begin", np.uint32),
                ("func_scope", np.uint32), ("instr_scope", np.uint32),
                ("scope_parent", np.uint32), ("scope_kind", np.uint8), ("scope_flags", np.uint8)]


def program_to_device(prog: dict, device="cuda"):
    """The descriptor arrays of `prog` as device tensors (uint32 arrays are
    carried as int32 tensors with the same bits)."""
    import torch
    out = dict(prog)
    for k, t in _DESC_FIELDS:
        a = np.ascontiguousarray(np.asarray(prog[k]), dtype=t)
        if t == np.uint32:
            a = a.view(np.int32)
        out[k] = torch.from_numpy(a.copy()).to(device)
    return out


def timing_enable(on: bool = True):
    """Device-time accounting per phase, with hipEvents on the caller's stream."""
    lib().gpa_timing_enable(int(bool(on)))


def timing_read(reset: bool = False) -> dict:
    ms = np.zeros(len(PHASES))
    calls = np.zeros(len(PHASES), np.uint64)
    lib().gpa_timing_read(ms.ctypes.data, calls.ctypes.data, len(PHASES), int(bool(reset)))
    return {name: (float(ms[k]), int(calls[k])) for k, name in enumerate(PHASES)}


class Program:
    """A program resident on the GPU with its static analysis."""

    def __init__(self, prog: dict, stream=None):
        L = lib()
        d = ProgramDesc()
        arrays = {}
        on_device = None
        for k, t in _DESC_FIELDS:
            a = prog[k]
            if isinstance(a, np.ndarray) or not hasattr(a, "data_ptr"):
                a = np.ascontiguousarray(np.asarray(a), dtype=t)
                dev = False
            else:
                dev = a.is_cuda
            if on_device is None:
                on_device = dev
            elif on_device != dev:
                raise ValueError("descriptor arrays must all be host or all be device arrays")
            arrays[k] = a
            setattr(d, k, _ptr(a))
        n = lambda k: int(arrays[k].shape[0])
        d.n_instr = n("op_class")
        d.n_blocks = n("block_begin") - 1
        d.n_funcs = n("func_block_begin") - 1
        d.n_scopes = n("scope_parent")
        d.n_regs, d.n_preds, d.n_bars = int(prog["n_regs"]), int(prog["n_preds"]), int(prog["n_bars"])
        d.on_device = int(bool(on_device))
        lat = np.asarray(prog["lat"], np.uint16)
        allowed = np.asarray(prog["allowed"], np.uint16)
        for i in range(16):
            d.arch.lat[i] = int(lat[i])
        for i in range(12):
            d.arch.allowed[i] = int(allowed[i])
        d.arch.blamable = int(prog["blamable"])
        self._arrays = arrays
        self.handle = ct.c_void_p()
        _check(L.gpa_load_program(ct.byref(d), _stream(stream), ct.byref(self.handle)))
        info = ProgramInfo()
        _check(L.gpa_program_get_info(self.handle, ct.byref(info)))
        self.info = {f: int(getattr(info, f)) for f, _ in ProgramInfo._fields_ if f != "pad"}
        self._arrays = None   # copied by the library

    def close(self):
        if getattr(self, "handle", None):
            lib().gpa_program_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def roots(self):
        """Kernel root scopes, ascending (the rows of Advice.topk)."""
        r = np.zeros(max(self.info["n_roots"], 1), np.uint32)
        _check(lib().gpa_program_roots(self.handle, r.ctypes.data))
        return r[:self.info["n_roots"]]

    def rd(self):
        i = self.info
        rd_ptr = np.zeros(i["n_uses"] + 1, np.uint32)
        rd_src = np.zeros(max(i["n_rd"], 1), np.uint32)
        rd_blk = np.zeros(max(i["n_rd"], 1), np.uint8)
        _check(lib().gpa_program_rd(self.handle, rd_ptr.ctypes.data, rd_src.ctypes.data,
                                    rd_blk.ctypes.data))
        return {"rd_ptr": rd_ptr, "rd_src": rd_src[:i["n_rd"]], "rd_blocked": rd_blk[:i["n_rd"]]}

    def edges(self):
        ne = self.info["n_edges"]
        m = max(ne, 1)
        src, dst = np.zeros(m, np.uint32), np.zeros(m, np.uint32)
        flags = np.zeros(m, np.uint8)
        dmin, dmax = np.zeros(m, np.uint32), np.zeros(m, np.uint32)
        _check(lib().gpa_program_edges(self.handle, src.ctypes.data, dst.ctypes.data,
                                       flags.ctypes.data, dmin.ctypes.data, dmax.ctypes.data))
        return {"src": src[:ne], "dst": dst[:ne], "flags": flags[:ne], "dmin": dmin[:ne],
                "dmax": dmax[:ne], "n_edges": ne}

    def attribute(self, samples, stream=None) -> "Blame":
        """`samples`: a numpy array of the 8-byte sample dtype (host), or a
        CUDA tensor whose bytes are the records (device)."""
        L = lib()
        if isinstance(samples, np.ndarray):
            a = np.ascontiguousarray(samples)
            n = a.nbytes // 8
            ptr, on_dev = a.ctypes.data, 0
        else:
            n = samples.numel() * samples.element_size() // 8
            ptr, on_dev = samples.data_ptr(), int(samples.is_cuda)
        h = ct.c_void_p()
        _check(L.gpa_attribute(self.handle, ptr if n else None, n, on_dev, _stream(stream),
                               ct.byref(h)))
        return Blame(self, h)


class Blame:
    def __init__(self, prog: Program, handle):
        self.prog = prog
        self.handle = handle

    def close(self):
        if getattr(self, "handle", None):
            lib().gpa_blame_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def counts(self):
        n = self.prog.info["n_instr"]
        C = np.zeros(n * 24, np.uint32)
        tot = np.zeros(4, np.uint64)
        _check(lib().gpa_blame_counts(self.handle, C.ctypes.data, tot.ctypes.data))
        return C.reshape(n, 12, 2), tot

    def shares(self):
        ne, nb = self.prog.info["n_edges"], self.prog.info["n_blamable"]
        s = np.zeros(max(ne * nb * 2, 1))
        _check(lib().gpa_blame_shares(self.handle, s.ctypes.data))
        return s[:ne * nb * 2].reshape(ne, nb, 2)

    def table(self):
        n = self.prog.info["n_instr"]
        b, s, f = np.zeros(n * 24), np.zeros(n * 24), np.zeros(n * N_FINE * 2)
        _check(lib().gpa_blame_table(self.handle, b.ctypes.data, s.ctypes.data, f.ctypes.data))
        return {"blamed": b.reshape(n, 12, 2), "self": s.reshape(n, 12, 2),
                "fine": f.reshape(n, N_FINE, 2)}

    def advise(self, stream=None) -> "Advice":
        h = ct.c_void_p()
        _check(lib().gpa_advise(self.handle, _stream(stream), ct.byref(h)))
        return Advice(self, h)


class Advice:
    def __init__(self, blame: Blame, handle):
        self.blame = blame
        self.handle = handle

    def close(self):
        if getattr(self, "handle", None):
            lib().gpa_advice_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get(self):
        ns = self.blame.prog.info["n_scopes"]
        act, mat, sp = np.zeros(ns), np.zeros(ns * N_OPT), np.zeros(ns * N_OPT)
        kT, kL, eq3 = np.zeros(ns), np.zeros(ns), np.zeros(ns * 3)
        _check(lib().gpa_advice_get(self.handle, act.ctypes.data, mat.ctypes.data, sp.ctypes.data,
                                    kT.ctypes.data, kL.ctypes.data, eq3.ctypes.data))
        return {"active": act, "matched": mat.reshape(ns, N_OPT), "speedup": sp.reshape(ns, N_OPT),
                "kernel_T": kT, "kernel_L": kL, "eq3": eq3.reshape(ns, 3)}

    def topk(self, k=5):
        """Rows in the order of Program.roots()."""
        ns = self.blame.prog.info["n_roots"]
        o, s = np.zeros(ns * k, np.uint32), np.zeros(ns * k, np.uint32)
        v = np.zeros(ns * k)
        _check(lib().gpa_advice_topk(self.handle, k, o.ctypes.data, s.ctypes.data, v.ctypes.data))
        return {"top_opt": o.reshape(ns, k), "top_scope": s.reshape(ns, k),
                "top_speed": v.reshape(ns, k)}
