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
          -4: "GPA_E_STATE", -5: "GPA_E_BUSY", -6: "GPA_E_UNSUPPORTED"}
GPA_E_BUSY = -5


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


class Launch(ct.Structure):
    _fields_ = [("blocks", ct.c_uint32), ("threads_per_block", ct.c_uint32),
                ("regs_per_thread", ct.c_uint32), ("shared_per_block", ct.c_uint32)]


class Device(ct.Structure):
    _fields_ = [(f, ct.c_uint32) for f in
                ("n_sm", "schedulers_per_sm", "warp_size", "max_warps_per_sm",
                 "max_blocks_per_sm", "max_threads_per_block", "regs_per_sm", "shared_per_sm")]


class ParallelEstimate(ct.Structure):
    _fields_ = [("matched", ct.c_uint32), ("pad", ct.c_uint32)] + \
               [(f, ct.c_double) for f in ("W", "W_new", "R_I", "I", "I_new", "C_W", "C_I", "f",
                                          "speedup")]


class Hotspot(ct.Structure):
    _fields_ = [("src", ct.c_uint32), ("dst", ct.c_uint32), ("dmin", ct.c_uint32),
                ("dmax", ct.c_uint32), ("samples", ct.c_double)]


class ServerStats(ct.Structure):
    _fields_ = [(f, ct.c_uint64) for f in
                ("submitted", "admitted", "completed", "failed", "batches", "max_batch",
                 "peak_reserved", "reserved", "budget", "queued", "inflight_batches")]


# every entry point declared in include/gpa.h
EXPORTS = ["gpa_load_program", "gpa_program_free", "gpa_program_get_info", "gpa_program_roots",
           "gpa_program_rd",
           "gpa_program_edges", "gpa_attribute", "gpa_blame_free", "gpa_blame_counts",
           "gpa_blame_shares", "gpa_blame_table", "gpa_advise", "gpa_advice_free",
           "gpa_advice_get", "gpa_advice_topk", "gpa_last_error", "gpa_timing_enable",
           "gpa_timing_read", "gpa_attribute_batch",
           "gpa_advise_batch", "gpa_pool_stats", "gpa_pool_trim", "gpa_server_create",
           "gpa_server_submit", "gpa_server_poll", "gpa_server_wait", "gpa_server_stats_get",
           "gpa_server_free",
           "gpa_parallel_advise", "gpa_program_coverage", "gpa_blame_hotspots", "gpa_report",
           "gpa_attribute_noalloc", "gpa_noalloc_scratch_bytes", "gpa_analyze_batch",
           "gpa_batch_free"]
PHASES = ["hist", "blame", "load", "advise", "rd_edges", "dist", "dfs", "rd_search",
          "validate", "sites", "edges", "targets", "dist_long"]

_lib = None


def _torch_runtime_first():
    """Bring up torch's HIP runtime before the library is loaded.

    torch ships its own HIP and HSA runtimes, and libgpa.so links the
    system's; a process that uses both holds two runtimes over one device.
    The library's runtime then finds the device only when it is loaded after
    torch's has come up (loaded first, its first call reports that no device
    is present), so the load order is fixed here."""
    try:
        import torch
    except ImportError:
        return
    if torch.cuda.is_available():
        torch.cuda.init()


def lib():
    """Load libgpa.so (built by paper_2009_04061_amd/build.py)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run paper_2009_04061_amd/build.py "
                              "(there is no fallback path)")
        _torch_runtime_first()
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
        L.gpa_attribute_batch.argtypes = [vp, vp, vp, u32, i32, vp, vp]
        L.gpa_attribute_batch.restype = ct.c_int32
        L.gpa_advise_batch.argtypes = [vp, u32, vp, vp]
        L.gpa_advise_batch.restype = ct.c_int32
        L.gpa_analyze_batch.argtypes = [vp, vp, vp, u32, i32, vp, vp, vp]
        L.gpa_analyze_batch.restype = ct.c_int32
        L.gpa_batch_free.argtypes = [vp, vp, u32]
        L.gpa_batch_free.restype = None
        L.gpa_parallel_advise.argtypes = [vp, u32, ct.POINTER(Launch), ct.POINTER(Device),
                                          ct.POINTER(ParallelEstimate)]
        L.gpa_parallel_advise.restype = ct.c_int32
        L.gpa_program_coverage.argtypes = [vp, vp, vp]
        L.gpa_blame_hotspots.argtypes = [vp, u32, u32, u32, vp, vp]
        L.gpa_report.argtypes = [vp, vp, u32, u32, vp, ct.POINTER(ct.c_size_t)]
        for name in ("gpa_program_coverage", "gpa_blame_hotspots", "gpa_report"):
            getattr(L, name).restype = ct.c_int32
        L.gpa_pool_stats.argtypes = [vp, vp]
        L.gpa_pool_trim.argtypes = []
        L.gpa_server_create.argtypes = [u64, pp]
        L.gpa_server_submit.argtypes = [vp, vp, vp, u64, i32, ct.POINTER(ct.c_uint64)]
        L.gpa_server_poll.argtypes = [vp, u64, pp, pp]
        L.gpa_server_wait.argtypes = [vp, u64, ct.POINTER(ct.c_uint64)]
        L.gpa_server_stats_get.argtypes = [vp, ct.POINTER(ServerStats)]
        L.gpa_server_free.argtypes = [vp]
        L.gpa_server_free.restype = None
        for name in ("gpa_pool_stats", "gpa_pool_trim", "gpa_server_create", "gpa_server_submit",
                     "gpa_server_poll", "gpa_server_wait", "gpa_server_stats_get"):
            getattr(L, name).restype = ct.c_int32
        L.gpa_noalloc_scratch_bytes.argtypes = []
        L.gpa_noalloc_scratch_bytes.restype = u64
        L.gpa_attribute_noalloc.argtypes = [vp, vp, u64, vp, vp, vp, vp, vp, vp, vp]
        L.gpa_attribute_noalloc.restype = ct.c_int32
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

    def coverage(self):
        """(single-dependency instructions before pruning, after pruning)."""
        a, b = ct.c_uint64(), ct.c_uint64()
        _check(lib().gpa_program_coverage(self.handle, ct.byref(a), ct.byref(b)))
        return int(a.value), int(b.value)

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

def noalloc_scratch_bytes() -> int:
    """gpa_noalloc_scratch_bytes: the fixed scratch of gpa_attribute_noalloc."""
    return int(lib().gpa_noalloc_scratch_bytes())


def attribute_noalloc(program, samples, counts, totals, share, blamed, self_, fine, stream=None):
    """gpa_attribute_noalloc: `samples` and the six outputs are CUDA tensors
    of the sizes include/gpa.h states; only enqueues work on `stream`."""
    n = samples.numel() * samples.element_size() // 8
    _check(lib().gpa_attribute_noalloc(program.handle, samples.data_ptr() if n else None, n,
                                       _stream(stream), counts.data_ptr(), totals.data_ptr(),
                                       share.data_ptr() if share is not None else None,
                                       blamed.data_ptr(), self_.data_ptr(), fine.data_ptr()))


def _records(samples):
    """(pointer, record count, on-device flag) of a sample array."""
    if isinstance(samples, np.ndarray):
        a = np.ascontiguousarray(samples)
        return a.ctypes.data, a.nbytes // 8, 0, a
    n = samples.numel() * samples.element_size() // 8
    return samples.data_ptr(), n, int(samples.is_cuda), samples


def attribute_batch(programs, samples, stream=None):
    """gpa_attribute_batch over (programs[k], samples[k]); all sample arrays
    on the host (numpy) or all on the device (CUDA tensors)."""
    count = len(programs)
    if len(samples) != count:
        raise ValueError("one sample array per program")
    recs = [_records(x) for x in samples]
    on_dev = {r[2] for r in recs}
    if len(on_dev) > 1:
        raise ValueError("sample arrays must all be host or all be device arrays")
    progs = (ct.c_void_p * max(count, 1))(*[p.handle for p in programs])
    ptrs = (ct.c_void_p * max(count, 1))(*[r[0] if r[1] else None for r in recs])
    ns = (ct.c_uint64 * max(count, 1))(*[r[1] for r in recs])
    out = (ct.c_void_p * max(count, 1))()
    _check(lib().gpa_attribute_batch(progs, ptrs, ns, count, on_dev.pop() if count else 1,
                                     _stream(stream), out))
    return [Blame(programs[k], ct.c_void_p(out[k])) for k in range(count)]


class BatchResult:
    """The handles of gpa_analyze_batch: blames[k] and advices[k] (Blame and
    Advice objects, made on first access, that do not free themselves);
    close() frees them all with gpa_batch_free."""

    def __init__(self, programs, bh, ah, count):
        self._programs, self._bh, self._ah, self._count = programs, bh, ah, count
        self._blames = self._advices = None

    @property
    def blames(self):
        if self._blames is None:
            self._blames = [Blame(self._programs[k], ct.c_void_p(self._bh[k]), owned=False)
                            for k in range(self._count)]
        return self._blames

    @property
    def advices(self):
        if self._advices is None:
            B = self.blames
            self._advices = [Advice(B[k], ct.c_void_p(self._ah[k]), owned=False)
                             for k in range(self._count)]
        return self._advices

    def close(self):
        if self._count is not None:
            lib().gpa_batch_free(self._bh, self._ah, self._count)
            for x in (self._blames or []) + (self._advices or []):
                x.handle = None
            self._count = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchInputs:
    """The argument arrays of a batched call (program handles, record
    pointers and counts), marshalled once for a batch that is analyzed
    repeatedly; the programs and sample arrays must outlive it."""

    def __init__(self, programs, samples):
        count = len(programs)
        if len(samples) != count:
            raise ValueError("one sample array per program")
        recs = [_records(x) for x in samples]
        on_dev = {r[2] for r in recs}
        if len(on_dev) > 1:
            raise ValueError("sample arrays must all be host or all be device arrays")
        self.programs, self.count = list(programs), count
        self.on_dev = on_dev.pop() if count else 1
        self._keep = [r[3] for r in recs]
        self.progs = (ct.c_void_p * max(count, 1))(*[p.handle for p in programs])
        self.ptrs = (ct.c_void_p * max(count, 1))(*[r[0] if r[1] else None for r in recs])
        self.ns = (ct.c_uint64 * max(count, 1))(*[r[1] for r in recs])


def analyze_batch(programs, samples=None, stream=None) -> BatchResult:
    """gpa_analyze_batch: attribute and advise every (programs[k],
    samples[k]) in one call; samples all host (numpy) or all device arrays.
    `programs` may instead be a BatchInputs (samples then None)."""
    inp = programs if isinstance(programs, BatchInputs) else BatchInputs(programs, samples)
    count = inp.count
    bh = (ct.c_void_p * max(count, 1))()
    ah = (ct.c_void_p * max(count, 1))()
    _check(lib().gpa_analyze_batch(inp.progs, inp.ptrs, inp.ns, count, inp.on_dev,
                                   _stream(stream), bh, ah))
    return BatchResult(inp.programs, bh, ah, count)


def advise_batch(blames, stream=None):
    """gpa_advise_batch over the blame handles."""
    count = len(blames)
    hs = (ct.c_void_p * max(count, 1))(*[b.handle for b in blames])
    out = (ct.c_void_p * max(count, 1))()
    _check(lib().gpa_advise_batch(hs, count, _stream(stream), out))
    return [Advice(blames[k], ct.c_void_p(out[k])) for k in range(count)]


class Blame:
    def __init__(self, prog: Program, handle, owned: bool = True):
        self.prog = prog
        self.handle = handle
        self.owned = owned   # False: freed with its batch (BatchResult.close)

    def close(self):
        if getattr(self, "handle", None):
            if self.owned:
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

    def parallel(self, root_index: int, launch: dict, device: dict):
        """gpa_parallel_advise: [Block Increase, Thread Increase] for the
        kernel root with index root_index (Program.roots() order)."""
        la = Launch(**{f: int(launch[f]) for f, _ in Launch._fields_})
        de = Device(**{f: int(device[f]) for f, _ in Device._fields_})
        out = (ParallelEstimate * 2)()
        _check(lib().gpa_parallel_advise(self.handle, int(root_index), ct.byref(la), ct.byref(de),
                                         out))
        return [{f: float(getattr(o, f)) for f, _ in ParallelEstimate._fields_ if f != "pad"}
                for o in out]

    def hotspots(self, root_index: int, opt: int, k: int = 5):
        """gpa_blame_hotspots: list of (src, dst, dmin, dmax, samples)."""
        out = (Hotspot * max(k, 1))()
        n = ct.c_uint32()
        _check(lib().gpa_blame_hotspots(self.handle, int(root_index), int(opt), int(k), out,
                                        ct.byref(n)))
        return [(o.src, o.dst, o.dmin, o.dmax, o.samples) for o in out[:n.value]]

    def advise(self, stream=None) -> "Advice":
        h = ct.c_void_p()
        _check(lib().gpa_advise(self.handle, _stream(stream), ct.byref(h)))
        return Advice(self, h)


class Advice:
    def __init__(self, blame: Blame, handle, owned: bool = True):
        self.blame = blame
        self.handle = handle
        self.owned = owned   # False: freed with its batch (BatchResult.close)

    def close(self):
        if getattr(self, "handle", None):
            if self.owned:
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


def pool_stats():
    """(bytes handed out, bytes cached) of the library's device pool."""
    a, b = ct.c_uint64(), ct.c_uint64()
    _check(lib().gpa_pool_stats(ct.byref(a), ct.byref(b)))
    return int(a.value), int(b.value)


def pool_trim():
    _check(lib().gpa_pool_trim())


class Server:
    """gpa_server_*: requests against resident programs, admitted by device
    bytes and run in batches by the library's worker thread."""

    def __init__(self, budget_bytes: int):
        self.handle = ct.c_void_p()
        _check(lib().gpa_server_create(int(budget_bytes), ct.byref(self.handle)))
        self._borrowed = {}    # ticket -> (program, samples): kept alive until polled

    def submit(self, program: Program, samples) -> int:
        ptr, n, on_dev, keep = _records(samples)
        t = ct.c_uint64()
        _check(lib().gpa_server_submit(self.handle, program.handle, ptr if n else None, n, on_dev,
                                       ct.byref(t)))
        self._borrowed[t.value] = (program, keep)
        return t.value

    def poll(self, ticket: int, want_blame: bool = False):
        """None while the request waits or runs; then (Advice, Blame or None)."""
        b, a = ct.c_void_p(), ct.c_void_p()
        st = lib().gpa_server_poll(self.handle, ticket, ct.byref(b) if want_blame else None,
                                   ct.byref(a))
        if st == GPA_E_BUSY:
            return None
        prog, _ = self._borrowed.pop(ticket, (None, None))
        _check(st)
        blame = Blame(prog, b) if want_blame else _Detached(prog)
        return Advice(blame, a), (blame if want_blame else None)

    def wait(self, timeout_s: float):
        """gpa_server_wait: the ticket of the next finished request (its
        results then poll without waiting), or None after timeout_s."""
        t = ct.c_uint64()
        st = lib().gpa_server_wait(self.handle, max(0, int(timeout_s * 1e6)), ct.byref(t))
        if st == GPA_E_BUSY:
            return None
        _check(st)
        return t.value

    def stats(self) -> dict:
        s = ServerStats()
        _check(lib().gpa_server_stats_get(self.handle, ct.byref(s)))
        return {f: int(getattr(s, f)) for f, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "handle", None):
            lib().gpa_server_free(self.handle)
            self.handle = None
            self._borrowed.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _Detached:
    """Stands in for a blame handle the server already freed (an Advice only
    needs its program)."""

    def __init__(self, prog):
        self.prog = prog
        self.handle = None


def report(advice: "Advice", blame: "Blame", top_optimizers: int = 5, hotspots: int = 5) -> str:
    """gpa_report: the advice as text."""
    n = ct.c_size_t(0)
    _check(lib().gpa_report(advice.handle, blame.handle, top_optimizers, hotspots, None,
                            ct.byref(n)))
    buf = ct.create_string_buffer(n.value)
    _check(lib().gpa_report(advice.handle, blame.handle, top_optimizers, hotspots, buf,
                            ct.byref(n)))
    return buf.value.decode()
