"""The batched path (gpa_attribute_batch, gpa_advise_batch) against the
per-profile path and the oracle.

Every profile of a batch must give bit for bit what gpa_attribute and
gpa_advise give for it alone (same kernels' arithmetic, same sum orders), and
sampled profiles are compared with the oracle element by element at the
tolerances of tests/parity.py."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2009_04061_amd import synth as S
from parity import compare, with_blamable

pytestmark = pytest.mark.gpu


def _outputs(P, B, A, k=16):
    C, tot = B.counts()
    out = {"C": C, "totals": tot, "shares": B.shares(), "table": B.table(), "est": A.get(),
           "top": A.topk(k), "roots": P.roots(), "info": P.info, "rd": P.rd(), "edges": P.edges()}
    return out


def _bitwise_equal(a, b, where):
    for key in ("C", "totals", "shares"):
        assert np.array_equal(np.asarray(a[key]).view(np.uint8), np.asarray(b[key]).view(np.uint8)), \
            (where, key)
    for grp in ("table", "est", "top"):
        for key in a[grp]:
            x, y = np.asarray(a[grp][key]), np.asarray(b[grp][key])
            assert x.shape == y.shape and np.array_equal(x.view(np.uint8), y.view(np.uint8)), \
                (where, grp, key)


def _device_records(torch, rec):
    raw = np.ascontiguousarray(rec).view(np.uint8)
    if raw.size == 0:
        return torch.zeros(0, dtype=torch.uint8, device="cuda")
    return torch.from_numpy(raw).cuda()


def _run_both(progs, recs, k=16, oracle_every=0, oracle_set=()):
    """Batch and per-profile runs of the same profiles: bitwise equal; the
    oracle on the chosen profiles."""
    import torch
    from paper_2009_04061_amd import gpa
    P = [gpa.Program(gpa.program_to_device(p)) for p in progs]
    D = [_device_records(torch, r) for r in recs]
    Bb = gpa.attribute_batch(P, D)
    Ab = gpa.advise_batch(Bb)
    checked = 0
    for i in range(len(progs)):
        b = _outputs(P[i], Bb[i], Ab[i], k)
        B1 = P[i].attribute(D[i])
        A1 = B1.advise()
        one = _outputs(P[i], B1, A1, k)
        _bitwise_equal(b, one, f"profile {i}")
        A1.close()
        B1.close()
        if i in oracle_set or (oracle_every and i % oracle_every == 0):
            print(f"oracle check of profile {i}: {len(progs[i]['op_class'])} instructions, "
                  f"{len(recs[i])} records", flush=True)
            o = O.run_all(progs[i], recs[i], k=k)
            compare(progs[i], b, o, k=k)
            checked += 1
        Ab[i].close()
        Bb[i].close()
    for p in P:
        p.close()
    return checked


def test_small_mixed_batch_equals_per_profile_and_oracle():
    """Mixed sizes, an empty profile, the same program in two entries, a
    profile whose records are not 16-byte aligned (counted by the plain
    path inside the batch call) and corrupted records."""
    import torch
    progs, recs = [], []
    for seed in range(10):
        prog = S.gen_program(seed=300 + seed, functions=[
            dict(n_instr=150 + 173 * seed, n_blocks=6 + 2 * seed, n_loops=2, max_depth=2,
                 kind="kernel"),
            dict(n_instr=60, n_blocks=3, n_loops=1, max_depth=1, kind="device")],
            n_regs=24, n_preds=4, n_bars=4, inline_frac=0.1)
        n = len(prog["op_class"])
        rec = S.gen_samples([0, 1, 7, 5000, 70_000, 130_001, 400_000, 3, 20_000, 1_000_003][seed],
                            n, 1.1, S.stall_mix_small(), seed=seed)
        progs.append(prog)
        recs.append(S.corrupt_samples(rec, 0.01, n, seed=seed) if seed % 3 == 0 else rec)
    progs.append(progs[4])
    recs.append(S.gen_samples(90_000, len(progs[4]["op_class"]), 1.2, S.stall_mix_small(), seed=99))
    assert _run_both(progs, recs, oracle_every=1) == len(progs)


def test_batch_of_mixed_blamable_sets():
    """Profiles whose architectures blame none, one, three and eleven
    reasons: the batch takes the twelve-slot blamer for all of them and
    must give what the four-slot one gives each profile alone."""
    progs, recs = [], []
    for i, mask in enumerate([None, 0, 1 << S.ST_SYNC, 0xFFE]):
        prog, rec = S.workload_small(seed=20 + i, n_samples=50_000)
        progs.append(prog if mask is None else with_blamable(prog, mask, seed=i))
        recs.append(rec)
    assert _run_both(progs, recs, oracle_every=1) == len(progs)


def test_unaligned_device_records_in_a_batch():
    import torch
    from paper_2009_04061_amd import gpa
    prog, rec = S.workload_small(seed=8, n_samples=60_000)
    P = gpa.Program(gpa.program_to_device(prog))
    raw = np.ascontiguousarray(rec).view(np.uint8)
    big = torch.zeros(raw.size + 8, dtype=torch.uint8, device="cuda")
    big[8:] = torch.from_numpy(raw).cuda()
    shifted = big[8:]                      # 8-byte aligned, not 16
    assert shifted.data_ptr() % 16 == 8
    Bb = gpa.attribute_batch([P, P], [shifted, _device_records(torch, rec)])
    Ab = gpa.advise_batch(Bb)
    B1 = P.attribute(_device_records(torch, rec))
    A1 = B1.advise()
    one = _outputs(P, B1, A1)
    for i in range(2):
        _bitwise_equal(_outputs(P, Bb[i], Ab[i]), one, f"entry {i}")
    o = O.run_all(prog, rec, k=16)
    compare(prog, one, o, k=16)


@pytest.mark.slow
def test_config2_full_batch_equals_per_profile():
    """The 1,024-profile batch at full size: every profile bitwise equal to
    its own per-profile run; the oracle on every 64th profile and on the
    largest ones."""
    progs, records, off = S.gen_batch(2)
    recs = [records[off[k]:off[k + 1]] for k in range(len(progs))]
    n_instr = np.array([len(p["op_class"]) for p in progs])
    largest = set(np.argsort(-n_instr)[:2].tolist()) | {int(np.argmax(np.diff(off)))}
    print(f"config 2: {len(progs)} profiles, {int(n_instr.sum())} instructions, "
          f"{int(off[-1])} records", flush=True)
    assert _run_both(progs, recs, oracle_every=64, oracle_set=largest) >= 16


@pytest.mark.slow
def test_config3_full_batch_equals_per_profile():
    """The whole-application batch at full size (400 kernels, 2M
    instructions, 500M records): every kernel bitwise equal to its own
    per-profile run; the oracle on every 40th kernel and the one with the
    most records."""
    progs, records, off = S.gen_batch(3)
    recs = [records[off[k]:off[k + 1]] for k in range(len(progs))]
    print(f"config 3: {len(progs)} kernels, {sum(len(p['op_class']) for p in progs)} "
          f"instructions, {int(off[-1])} records", flush=True)
    most = {int(np.argmax(np.diff(off)))}
    assert _run_both(progs, recs, oracle_every=40, oracle_set=most) >= 10


def test_analyze_batch_equals_attribute_then_advise_batch():
    """gpa_analyze_batch (one call, no return to the host between the blamer
    and the estimators) against gpa_attribute_batch + gpa_advise_batch: bit
    for bit, on a mixed batch with an empty and an unaligned entry."""
    import torch
    from paper_2009_04061_amd import gpa
    progs, recs = [], []
    for seed in range(5):
        prog, rec = S.workload_small(seed=500 + seed, n_samples=[0, 3, 40_000, 250_000, 900_001][seed])
        progs.append(prog)
        recs.append(rec)
    P = [gpa.Program(gpa.program_to_device(p)) for p in progs]
    D = [_device_records(torch, r) for r in recs]
    raw = np.ascontiguousarray(recs[3]).view(np.uint8)
    big = torch.zeros(raw.size + 8, dtype=torch.uint8, device="cuda")
    big[8:] = torch.from_numpy(raw.copy()).cuda()
    D[3] = big[8:]
    R = gpa.analyze_batch(P, D)
    Bb = gpa.attribute_batch(P, D)
    Ab = gpa.advise_batch(Bb)
    for i in range(len(P)):
        _bitwise_equal(_outputs(P[i], R.blames[i], R.advices[i]), _outputs(P[i], Bb[i], Ab[i]),
                       f"profile {i}")
        Ab[i].close()
        Bb[i].close()
    R.close()
    for p in P:
        p.close()
