"""gpa_attribute_noalloc (the histogram and blamer with fixed device
scratch, for callers that cannot allocate) against gpa_attribute, called
through the C-ABI: counts, totals, shares and the per-instruction tables
must be bit for bit the same, on two calls in a row with the second one
smaller, and the call must take nothing from the library's allocator."""
import ctypes as ct

import numpy as np
import pytest

from paper_2009_04061_amd import synth as S

pytestmark = pytest.mark.gpu

N_FINE = 8


def _abi():
    from paper_2009_04061_amd import gpa
    return gpa, gpa.lib()


def _pool_in_use(L):
    a, b = ct.c_uint64(), ct.c_uint64()
    assert L.gpa_pool_stats(ct.byref(a), ct.byref(b)) == 0
    return a.value


def _noalloc(gpa, L, P, dev_rec, stream=None):
    import torch
    info = P.info
    ni, ne, nb = info["n_instr"], info["n_edges"], info["n_blamable"]
    out = {"counts": torch.full((ni * 24,), 0x5A5A5A5A, dtype=torch.int32, device="cuda"),
           "totals": torch.full((4,), -1, dtype=torch.int64, device="cuda"),
           "share": torch.full((max(ne * nb * 2, 1),), float("nan"), dtype=torch.float64,
                               device="cuda"),
           "blamed": torch.full((ni * 24,), float("nan"), dtype=torch.float64, device="cuda"),
           "self": torch.full((ni * 24,), float("nan"), dtype=torch.float64, device="cuda"),
           "fine": torch.full((ni * N_FINE * 2,), float("nan"), dtype=torch.float64,
                              device="cuda")}
    torch.cuda.synchronize()
    n = dev_rec.numel() // 8
    before = _pool_in_use(L)
    st = L.gpa_attribute_noalloc(P.handle, dev_rec.data_ptr() if n else None, n,
                                 gpa._stream(stream), out["counts"].data_ptr(),
                                 out["totals"].data_ptr(), out["share"].data_ptr(),
                                 out["blamed"].data_ptr(), out["self"].data_ptr(),
                                 out["fine"].data_ptr())
    assert st == 0, L.gpa_last_error().decode()
    torch.cuda.synchronize()
    assert _pool_in_use(L) == before, "the no-allocation call took memory from the pool"
    return {"C": out["counts"].cpu().numpy().view(np.uint32).reshape(ni, 12, 2),
            "totals": out["totals"].cpu().numpy().view(np.uint64),
            "shares": out["share"].cpu().numpy()[:ne * nb * 2].reshape(ne, nb, 2),
            "blamed": out["blamed"].cpu().numpy().reshape(ni, 12, 2),
            "self": out["self"].cpu().numpy().reshape(ni, 12, 2),
            "fine": out["fine"].cpu().numpy().reshape(ni, N_FINE, 2)}


def _plain(P, dev_rec):
    B = P.attribute(dev_rec)
    C, tot = B.counts()
    t = B.table()
    r = {"C": C, "totals": tot, "shares": B.shares(), "blamed": t["blamed"], "self": t["self"],
         "fine": t["fine"]}
    B.close()
    return r


def _same(a, b, where):
    for key in ("C", "totals", "shares", "blamed", "self", "fine"):
        x, y = np.ascontiguousarray(a[key]), np.ascontiguousarray(b[key])
        assert x.shape == y.shape and np.array_equal(x.view(np.uint8), y.view(np.uint8)), \
            (where, key)


def _dev(rec):
    import torch
    return torch.from_numpy(np.ascontiguousarray(rec).view(np.uint8).copy()).cuda()


def test_noalloc_equals_attribute_on_two_calls_the_second_smaller():
    gpa, L = _abi()
    prog, rec = S.workload_small(seed=3, n_samples=300_000)
    P = gpa.Program(gpa.program_to_device(prog))
    big = _dev(rec)
    small = _dev(S.corrupt_samples(rec[:70_001], 0.01, len(prog["op_class"]), seed=4))
    print("no-alloc call 1: 300,000 records", flush=True)
    _same(_noalloc(gpa, L, P, big), _plain(P, big), "first call")
    print("no-alloc call 2: 70,001 records", flush=True)
    _same(_noalloc(gpa, L, P, small), _plain(P, small), "second, smaller call")
    P.close()


def test_noalloc_on_the_large_profile_and_an_empty_one():
    gpa, L = _abi()
    prog, rec = S.workload_large(seed=1, n_samples=20_000_000)
    P = gpa.Program(gpa.program_to_device(prog))
    d = _dev(rec)
    print("no-alloc call: large profile, 20M records", flush=True)
    _same(_noalloc(gpa, L, P, d), _plain(P, d), "large profile")
    import torch
    empty = torch.zeros(0, dtype=torch.uint8, device="cuda")
    print("no-alloc call: no records", flush=True)
    _same(_noalloc(gpa, L, P, empty), _plain(P, empty), "empty profile")
    P.close()


def _outputs_for(P):
    import torch
    info = P.info
    ni, ne, nb = info["n_instr"], info["n_edges"], info["n_blamable"]
    return [torch.zeros(ni * 24, dtype=torch.int32, device="cuda"),
            torch.zeros(4, dtype=torch.int64, device="cuda"),
            torch.zeros(max(ne * nb * 2, 1), dtype=torch.float64, device="cuda"),
            torch.zeros(ni * 24, dtype=torch.float64, device="cuda"),
            torch.zeros(ni * 24, dtype=torch.float64, device="cuda"),
            torch.zeros(ni * N_FINE * 2, dtype=torch.float64, device="cuda")]


def test_noalloc_rejects_inputs_beyond_its_scratch():
    """Checked on the host before any launch: GPA_E_UNSUPPORTED with a
    message, and the library stays usable.  The refused call gets a record
    buffer of its full size and output arrays of theirs, so that nothing
    would be read or written out of bounds even if the check let it through.
    The program has more than 3,072 instructions, so its histogram keeps cold
    keys (8 bytes of scratch per record); a smaller program's scratch does
    not grow with the records."""
    import torch
    gpa, L = _abi()
    prog, rec = S.workload_large(seed=1, n_samples=2_000_000)
    P = gpa.Program(gpa.program_to_device(prog))
    cap = L.gpa_noalloc_scratch_bytes()
    n_too_many = cap // 8 + 1   # the cold-key arrays alone take 8 bytes per record
    big = torch.zeros(n_too_many * 8, dtype=torch.uint8, device="cuda")
    outs = _outputs_for(P)
    torch.cuda.synchronize()
    st = L.gpa_attribute_noalloc(P.handle, big.data_ptr(), n_too_many, None,
                                 *[t.data_ptr() for t in outs])
    assert st == -6 and b"scratch" in L.gpa_last_error()
    del big
    d = _dev(rec)
    _same(_noalloc(gpa, L, P, d), _plain(P, d), "after the refused call")
    P.close()
