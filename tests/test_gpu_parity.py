"""GPU parity: the HIP path through the C-ABI against the oracle, element by
element on the same seeded inputs."""
import numpy as np
import pytest

import brute as B
from asm import assemble, samples
from oracle import oracle as O
from paper_2009_04061_amd import synth as S
from parity import compare, run_gpu, with_blamable

pytestmark = pytest.mark.gpu


def _both(prog, rec, k=16, **kw):
    # k = 16, the largest the library takes: kernels with fewer candidates
    # than k end their rows with empty entries on both sides
    g = run_gpu(prog, rec, k=k, **kw)
    o = O.run_all(prog, rec, k=k)
    compare(prog, g, o, k=k)
    return g, o


def test_small_workload_full_parity():
    prog, rec = S.workload_small(seed=0)
    g, o = _both(prog, rec)
    assert g["info"]["n_edges"] > 1000


def test_host_inputs_match_device_inputs():
    prog, rec = S.workload_small(seed=11, n_samples=50_000)
    g = run_gpu(prog, rec, device_inputs=False)
    o = O.run_all(prog, rec)
    compare(prog, g, o)


def test_multi_kernel_device_and_math_functions():
    prog, rec = S.workload_multi(seed=7, n_samples=150_000)
    _both(prog, rec)


@pytest.mark.parametrize("seed", range(12))
def test_random_arbitrary_cfgs(seed):
    """Arbitrary (irreducible, partly unreachable) tiny CFGs with random
    guards, complementary pairs, barriers and read barriers."""
    prog = B.random_cfg_program(seed, n_blocks=int(3 + seed % 6), max_block=5, n_locs=4)
    n = len(prog["op_class"])
    rec = S.gen_samples(5000, n, 0.8, S.stall_mix_small(), seed=seed)
    _both(prog, rec)


@pytest.mark.parametrize("seed", range(6))
def test_random_structured_programs(seed):
    prog = S.gen_program(seed=100 + seed, functions=[
        dict(n_instr=300 + 50 * seed, n_blocks=20 + 3 * seed, n_loops=4, max_depth=3, kind="kernel"),
        dict(n_instr=80, n_blocks=6, n_loops=1, max_depth=1, kind="device")],
        n_regs=12, n_preds=3, n_bars=4, guard_frac=0.3, pair_frac=0.15, inline_frac=0.1)
    n = len(prog["op_class"])
    rec = S.gen_samples(40_000, n, 1.0, S.stall_mix_small(), seed=seed)
    _both(prog, rec)


def test_dropped_records_and_ragged_tail():
    prog, rec = S.workload_small(seed=4, n_samples=3 * 16384 + 77)
    bad = S.corrupt_samples(rec, 0.03, 2000, seed=9)
    g, o = _both(prog, bad)
    assert g["totals"][2] > 0


def test_empty_and_single_sample():
    prog, _ = S.workload_small(seed=5, n_samples=10)
    _both(prog, np.zeros(0, S.SAMPLE_DTYPE))
    _both(prog, samples([(17, S.ST_MEM_DEP, 1, 1)]))


def test_worked_examples_on_gpu():
    prog = assemble("block 0 ->\n  @!P0 LDC R0 <- R5\n  MOV R7 <- R8\n  @P0 LDG R0 <- R2 R3\n"
                    "  MOV R9 <- R8\n  IADD R1 <- R0 R6\n")
    rec = samples([(0, S.ST_SELECTED, 0, 8), (2, S.ST_SELECTED, 0, 4), (4, S.ST_MEM_DEP, 1, 10)])
    g, _ = _both(prog, rec)
    assert g["table"]["blamed"][0, S.ST_MEM_DEP, 1] == 5.0
    assert g["table"]["blamed"][2, S.ST_MEM_DEP, 1] == 5.0


def _long_search_program(n=120):
    """A loop of n blocks where every block branches to the next two: a use
    at the latch reaches back over the whole loop to the defs before it, so
    its backward search meets far more blocks than one thread keeps track of
    (the workgroup search takes it).  R0 has one plain and one guarded def,
    R2 a complementary pair, R10 a def after the loop only; one block in the
    middle reads R0 unpredicated (dominator pruning cuts there)."""
    lines = ["block 0 -> 1", "  MOV R0 <- R1", "  @P0 MOV R2 <- R1", "  @!P0 MOV R2 <- R3"]
    for b in range(1, n):
        succ = [b + 1] if b + 1 < n else [1, n]
        if b + 2 < n:
            succ.append(b + 2)
        lines.append(f"block {b} -> " + " ".join(map(str, succ)))
        if b == n // 2:
            lines.append("  IADD R4 <- R0 R5")
        elif b % 7 == 0:
            lines.append("  @P1 MOV R0 <- R6")
        else:
            lines.append(f"  IADD R{7 + b % 3} <- R{11 + b % 3}")
        if b == n - 1:
            lines.append("  IADD R5 <- R0 R2")
            lines.append("  @P1 IADD R6 <- R10 R0")
        lines.append("  BRA")
    lines += [f"block {n} ->", "  MOV R10 <- R0", f"loop 1 {n - 1}"]
    return assemble("\n".join(lines) + "\n")


def test_long_backward_searches():
    prog = _long_search_program()
    o = O.Program(prog)
    # some use is reached by defs from all around the loop
    assert max(len(o.sources(u)) for u in range(o.n_uses)) >= 10
    n = len(prog["op_class"])
    rec = S.gen_samples(20_000, n, 0.7, S.stall_mix_small(), seed=21)
    _both(prog, rec)


def _hub_program(k):
    """One block defines R5 and branches to k blocks, each reading R5 and
    defining R0; they join in a block that reads R0.  The join's use has k
    incoming edges and R5's def k + 1 outgoing ones, so with k > 64 one
    destination's (and one source's) edges span several 64-edge chunks of
    the blamer's wave tiles."""
    lines = ["block 0 -> " + " ".join(str(i) for i in range(1, k + 1)), "  MOV R5 <- R1", "  BRA"]
    for i in range(1, k + 1):
        lines += [f"block {i} -> {k + 1}", "  MOV R0 <- R5", "  BRA"]
    lines += [f"block {k + 1} ->", "  IADD R2 <- R0 R3", "  IADD R4 <- R2 R5"]
    return assemble("\n".join(lines) + "\n")


@pytest.mark.parametrize("k", [63, 64, 65, 150])
def test_high_in_and_out_degree(k):
    prog = _hub_program(k)
    o = O.Program(prog)
    a = o.analyze()
    n = len(prog["op_class"])
    assert np.bincount(a["dst"], minlength=n).max() == k
    assert np.bincount(a["src"], minlength=n).max() == k + 1
    rec = S.gen_samples(50_000, n, 0.5, S.stall_mix_small(), seed=k)
    _both(prog, rec)


# no blamable reason; one (the four-slot kernels); eleven and all twelve
# (the twelve-slot kernels, with the issued reason itself blamable)
@pytest.mark.parametrize("mask", [0, 1 << S.ST_SYNC, 0xFFE, 0xFFF])
def test_blamable_sets_of_other_architectures(mask):
    prog, rec = S.workload_small(seed=5, n_samples=80_000)
    p = with_blamable(prog, mask, seed=5)
    g, _ = _both(p, rec)
    assert g["info"]["n_blamable"] == bin(mask).count("1")


def test_deterministic_bitwise():
    prog, rec = S.workload_multi(seed=3, n_samples=60_000)
    a = run_gpu(prog, rec)
    b = run_gpu(prog, rec)
    for key in ("shares",):
        assert np.array_equal(a[key], b[key])
    for key in ("blamed", "self", "fine"):
        assert np.array_equal(a["table"][key], b["table"][key])
    for key in ("matched", "speedup", "active"):
        assert np.array_equal(a["est"][key], b["est"][key])


def test_large_workload_full_parity():
    """The 60k-instruction, 1,500-block profile with 20M samples, compared
    in full (the oracle finishes it in seconds)."""
    import time
    t = time.time()
    prog, rec = S.workload_large(seed=1)
    print(f"\n  generated in {time.time() - t:.1f}s", flush=True)
    # k = 16, the largest the library takes: every selection round is checked
    g = run_gpu(prog, rec, k=16)
    print(f"  gpu done at {time.time() - t:.1f}s", flush=True)
    o = O.run_all(prog, rec, k=16)
    print(f"  oracle done at {time.time() - t:.1f}s", flush=True)
    compare(prog, g, o, k=16)
    assert g["info"]["n_edges"] > 100_000


def test_program_past_16_bit_walks():
    """70,000 instructions in one function: walks can pass 65,533
    instructions, so the walk tables keep 32-bit entries."""
    prog = S.gen_program(seed=31, functions=[dict(n_instr=70_000, n_blocks=900, n_loops=40,
                                                  max_depth=4, kind="kernel")],
                         n_regs=64, n_preds=4, n_bars=8)
    n = len(prog["op_class"])
    assert n >= 0xFFFE
    rec = S.gen_samples(300_000, n, 1.1, S.stall_mix_small(), seed=31)
    _both(prog, rec)


def test_function_at_block_limit_and_beyond():
    from paper_2009_04061_amd import gpa
    ok = S.gen_program(seed=8, functions=[dict(n_instr=4096 * 2, n_blocks=4096, n_loops=20,
                                               max_depth=3, kind="kernel")],
                       n_regs=32, n_preds=4, n_bars=4)
    rec = S.gen_samples(100_000, 8192, 1.1, S.stall_mix_small(), seed=8)
    _both(ok, rec)
    big = S.gen_program(seed=9, functions=[dict(n_instr=4097 * 2, n_blocks=4097, n_loops=5,
                                                max_depth=2, kind="kernel")],
                        n_regs=32, n_preds=4, n_bars=4)
    with pytest.raises(gpa.GpaError) as ei:
        gpa.Program(big)
    assert ei.value.status == -6


def _corrupt(prog, kind):
    """A copy of `prog` with one malformed field; every array keeps its
    declared size, so only the library's own checks can reject it."""
    q = {k: (np.array(v, copy=True) if isinstance(v, np.ndarray) else v) for k, v in prog.items()}
    nb = len(q["block_begin"]) - 1
    ns = len(q["scope_parent"])
    n_loc = q["n_regs"] + q["n_preds"] + q["n_bars"]
    if kind == "succ_target":
        q["succ"][len(q["succ"]) // 2] = nb + 5
    elif kind == "block_order":
        q["block_begin"][3] = q["block_begin"][4] + 1
    elif kind == "def_loc":
        q["def_loc"][7] = n_loc + 2
    elif kind == "instr_scope":
        q["instr_scope"][11] = ns + 3
    elif kind == "scope_parent":
        q["scope_parent"][ns - 1] = ns - 1
    elif kind == "guard":
        q["guard"][5] = 2 * q["n_preds"] + 1
    elif kind == "op_class":
        q["op_class"][9] = 200
    elif kind == "def_csr":
        q["def_ptr"][20] = q["def_ptr"][21] + 1
    elif kind == "func_bounds":
        q["func_block_begin"][1] = q["func_block_begin"][2]
    return q


@pytest.mark.parametrize("kind", ["succ_target", "block_order", "def_loc", "instr_scope",
                                  "scope_parent", "guard", "op_class", "def_csr", "func_bounds"])
def test_malformed_descriptor_is_rejected(kind):
    from paper_2009_04061_amd import gpa
    prog, _ = S.workload_multi(seed=3, n_samples=10)
    assert len(prog["func_block_begin"]) > 3
    print(f"  malformed descriptor: {kind}", flush=True)
    with pytest.raises(gpa.GpaError) as ei:
        gpa.Program(_corrupt(prog, kind))
    assert ei.value.status == -1, kind
    # the library is still usable after a rejected load
    P = gpa.Program(prog)
    assert P.info["n_edges"] > 0
    P.close()


def _hist_only(P, prog, rec, offset_bytes=0):
    """Counts and totals of one gpa_attribute call against the oracle's
    histogram; `offset_bytes` places the device records at that offset from
    a 256-byte aligned allocation."""
    import torch
    raw = np.ascontiguousarray(rec).view(np.uint8)
    buf = torch.zeros(raw.size + offset_bytes, dtype=torch.uint8, device="cuda")
    buf[offset_bytes:] = torch.from_numpy(raw.copy()).cuda()
    B = P.attribute(buf[offset_bytes:])
    C, tot = B.counts()
    B.close()
    Co, dropped = O.count(len(prog["op_class"]), rec)
    from parity import _equal
    _equal(C, Co, "counts")
    _equal(int(tot[0]), int(Co.sum()), "valid samples")
    _equal(int(tot[1]), int(Co[:, :, 1].sum()), "latency samples")
    _equal(int(tot[2]), dropped, "dropped records")


@pytest.fixture(scope="module")
def large_program():
    from paper_2009_04061_amd import gpa
    prog, rec = S.workload_large(seed=1)
    P = gpa.Program(gpa.program_to_device(prog))
    yield prog, rec, P
    P.close()


def test_histogram_hot_and_cold_extremes(large_program):
    """The hot-set histogram: uniform PCs over 60k instructions (almost every
    record cold: a workgroup stages and flushes its cold keys many times),
    one PC only (all hot), a flat head of 3,000 PCs (more candidates than hot
    slots), invalid records, and records 8 bytes off 16-byte alignment."""
    prog, _, P = large_program
    n_instr = len(prog["op_class"])
    rng = np.random.default_rng(12)
    mix = S.stall_mix_small()
    uni = S.gen_samples(20_000_000, n_instr, 0.0, mix, seed=12)
    uni["pc"] = rng.integers(0, n_instr, len(uni))
    print("  uniform", flush=True)
    _hist_only(P, prog, S.corrupt_samples(uni, 0.001, n_instr, seed=12))
    one = S.gen_samples(1_000_003, n_instr, 0.0, mix, seed=13)
    one["pc"] = 4242
    print("  one pc", flush=True)
    _hist_only(P, prog, one)
    flat = S.gen_samples(3_000_001, n_instr, 0.0, mix, seed=14)
    flat["pc"] = rng.permutation(n_instr)[:3000][rng.integers(0, 3000, len(flat))]
    print("  flat head, misaligned", flush=True)
    _hist_only(P, prog, S.corrupt_samples(flat, 0.01, n_instr, seed=14), offset_bytes=8)


@pytest.mark.parametrize("path", ["hot", "partition"])
def test_histogram_paths_on_the_large_profile(large_program, monkeypatch, path):
    """The 20M-record Zipf profile through either histogram path (the
    partition path serves programs beyond the hot path's PC range, and is
    forced here), aligned and 8 bytes off."""
    prog, rec, P = large_program
    if path == "partition":
        monkeypatch.setenv("GPA_HIST_PARTITION", "1")
    _hist_only(P, prog, rec)
    _hist_only(P, prog, rec[: len(rec) - 5], offset_bytes=8)


def test_histogram_bucket_outgrows_its_estimate(monkeypatch):
    """Records of one bucket placed only where the size estimate does not look
    (every slice of 512 records except each 32nd), so its runs overflow their
    regions and go the overflow way; the other slices feed a bucket of their
    own, and a few invalid records are mixed in."""
    prog, _ = S.workload_small(seed=6, n_samples=10)
    n = 1_500_000
    rng = np.random.default_rng(6)
    rec = np.zeros(n, S.SAMPLE_DTYPE)
    pos = np.arange(n)
    sampled = (pos // 512) % 32 == 0
    rec["pc"][sampled] = rng.integers(0, 512, int(sampled.sum()))
    hot = rng.random(n) < 0.6
    rec["pc"][~sampled] = np.where(hot[~sampled], 1100, rng.integers(1024, 1536, int((~sampled).sum())))
    rec["stall"] = rng.integers(0, 12, n)
    rec["flags"] = (rng.random(n) < 0.5) & (rec["stall"] != S.ST_SELECTED) & (rec["stall"] != S.ST_NOT_SELECTED)
    rec = S.corrupt_samples(rec, 0.001, len(prog["op_class"]), seed=6)
    print(f"  records {n}, sampled slices {int(sampled.sum())}", flush=True)
    monkeypatch.setenv("GPA_HIST_PARTITION", "1")   # the sizing belongs to the partition path
    _both(prog, rec)
    monkeypatch.delenv("GPA_HIST_PARTITION")
    _both(prog, rec)


def _one_bin(n, pc, stall, lam):
    rec = np.zeros(n, S.SAMPLE_DTYPE)
    rec["pc"] = pc
    rec["stall"] = stall
    rec["flags"] = lam
    return rec


def test_direct_histogram_counter_wraps():
    """The direct mode (every bin of a program of at most 3,072 instructions
    in LDS, two 16-bit counters per word): one bin taking far more than
    2^16 records per workgroup range, in both counters of a word, and the
    double wrap (the low counter wraps into a high counter that holds
    0xFFFF); exact against the oracle's counts."""
    from paper_2009_04061_amd import gpa
    prog, _ = S.workload_small(seed=7, n_samples=10)
    P = gpa.Program(gpa.program_to_device(prog))
    rng = np.random.default_rng(7)
    mem = S.STALL_NAMES.index("MEM_DEP")
    # 700k low-counter and 450k high-counter records of one word, shuffled,
    # with a light background
    rec = np.concatenate([_one_bin(700_000, 5, mem, 0), _one_bin(450_000, 5, mem, 1),
                          S.gen_samples(50_000, len(prog["op_class"]), 1.1, S.stall_mix_small(),
                                        seed=7)])
    rec = rec[rng.permutation(len(rec))]
    print("  one word, both counters", flush=True)
    _hist_only(P, prog, rec)
    # 65,535 high-counter records, then 65,536 low ones: the last low record
    # wraps both counters of the word (one range: 131,071 records)
    dbl = np.concatenate([_one_bin(65_535, 9, mem, 1), _one_bin(65_536, 9, mem, 0)])
    print("  double wrap", flush=True)
    _hist_only(P, prog, dbl)
    _hist_only(P, prog, dbl[::-1].copy())
    # the same through the batched path, in one batch with an ordinary profile
    B = gpa.attribute_batch([P, P], [_dev(rec), _dev(dbl)])
    for b, r in zip(B, (rec, dbl)):
        C, tot = b.counts()
        Co, dropped = O.count(len(prog["op_class"]), r)
        from parity import _equal
        _equal(C, Co, "batched counts")
        _equal(int(tot[0]), int(Co.sum()), "batched valid samples")
        _equal(int(tot[1]), int(Co[:, :, 1].sum()), "batched latency samples")
        b.close()
    P.close()


def _dev(rec):
    import torch
    return torch.from_numpy(np.ascontiguousarray(rec).view(np.uint8).copy()).cuda()


@pytest.mark.parametrize("seed", range(3))
def test_small_programs_through_the_hot_and_cold_path(monkeypatch, seed):
    """Programs small enough for the direct mode, forced through the
    hot-set / cold-key path instead (GPA_HIST_HOTSET=1): whole-path parity,
    so that both histogram modes stay covered on small programs."""
    monkeypatch.setenv("GPA_HIST_HOTSET", "1")
    prog, rec = S.workload_small(seed=40 + seed, n_samples=[200_000, 1_000_003, 37][seed])
    _both(prog, S.corrupt_samples(rec, 0.01, len(prog["op_class"]), seed=seed))


def _golden_cases():
    import json
    import os
    gold = os.path.join(os.path.dirname(__file__), "golden")
    for name in sorted(os.listdir(gold)):
        with open(os.path.join(gold, name)) as f:
            g = json.load(f)
        if "program" in g and "samples" in g:
            yield name, g["program"], g["samples"]
        for k, c in enumerate(g.get("cases", [])):
            text = c.get("program", g.get("program"))
            if text is not None and "samples" in c:
                yield f"{name}[{k}]", text, c["samples"]


GOLDEN = list(_golden_cases())


@pytest.mark.parametrize("name,text,spec", GOLDEN, ids=[g[0] for g in GOLDEN])
def test_hand_worked_programs_on_gpu(name, text, spec):
    """Every hand-worked program of tests/golden (Table 2 rows, Fig. 5 fine
    classes, Eq. (3), ranking ties, saturated estimates) through the HIP
    path, element by element against the oracle."""
    prog = assemble(text)
    rec = samples([(pc, S.STALL_NAMES.index(st), lam, n) for pc, st, lam, n in spec])
    _both(prog, rec)


def _parallel_close(g, o, where):
    for key in ("matched", "W", "W_new", "R_I", "I", "I_new", "C_W", "C_I", "f", "speedup"):
        assert g[key] == pytest.approx(o[key], rel=1e-12, abs=1e-15), (where, key)


def test_parallel_estimators_on_gpu():
    """gpa_parallel_advise against the oracle: the hand-worked launches of
    tests/golden, and every kernel root of the multi-kernel workload under a
    few launches and devices."""
    import json
    import os
    from paper_2009_04061_amd import gpa
    with open(os.path.join(os.path.dirname(__file__), "golden", "parallel_estimators.json")) as f:
        g = json.load(f)
    prog = assemble(g["program"])
    for c in g["cases"]:
        rec = samples([(pc, S.STALL_NAMES.index(st), lam, n) for pc, st, lam, n in c["samples"]])
        P = gpa.Program(prog)
        B = P.attribute(rec)
        got = B.parallel(0, c["launch"], g["device"])
        Po = O.Program(prog)
        C, _ = O.count(Po.n_instr, rec)
        want = O.parallel(Po, C, 0, c["launch"], g["device"])
        for k in range(2):
            _parallel_close(got[k], want[k], (c["name"], k))
        B.close()
        P.close()
    prog, rec = S.workload_multi(seed=9, n_samples=120_000)
    P = gpa.Program(gpa.program_to_device(prog))
    B = P.attribute(rec)
    Po = O.Program(prog)
    C, _ = O.count(Po.n_instr, rec)
    mi355x = {"n_sm": 256, "schedulers_per_sm": 4, "warp_size": 64, "max_warps_per_sm": 32,
              "max_blocks_per_sm": 32, "max_threads_per_block": 1024, "regs_per_sm": 4 * 512 * 64,
              "shared_per_sm": 160 * 1024}
    launches = [dict(blocks=100, threads_per_block=256, regs_per_thread=64, shared_per_block=0),
                dict(blocks=100000, threads_per_block=64, regs_per_thread=0, shared_per_block=0),
                dict(blocks=3, threads_per_block=64, regs_per_thread=0, shared_per_block=4096)]
    for ri, root in enumerate(P.roots()):
        for li, la in enumerate(launches):
            got = B.parallel(ri, la, mi355x)
            want = O.parallel(Po, C, int(root), la, mi355x)
            for k in range(2):
                _parallel_close(got[k], want[k], (int(root), li, k))
    B.close()
    P.close()


def _hotspots_match(got, want, where):
    assert len(got) == len(want), (where, got, want)
    for g_, w in zip(got, want):
        if g_[:4] != w[:4]:
            # a tie within rounding may order two carriers either way
            assert abs(g_[4] - w[4]) <= 1e-9 * max(1.0, abs(w[4])), (where, g_, w)
        assert g_[4] == pytest.approx(w[4], rel=1e-12), (where, g_, w)


@pytest.mark.parametrize("which", ["small", "multi", "golden"])
def test_report_coverage_and_hotspots_on_gpu(which):
    """Single dependency coverage and every optimizer's top hotspots per
    kernel against the oracle; the text report is produced."""
    import json
    import os
    from paper_2009_04061_amd import gpa
    if which == "small":
        prog, rec = S.workload_small(seed=2, n_samples=150_000)
    elif which == "multi":
        prog, rec = S.workload_multi(seed=3, n_samples=150_000)
    else:
        with open(os.path.join(os.path.dirname(__file__), "golden", "report_coverage.json")) as f:
            g = json.load(f)
        prog = assemble(g["program"])
        rec = samples([(19, S.ST_MEM_DEP, 1, 7), (18, S.ST_SELECTED, 0, 2)])
    P = gpa.Program(gpa.program_to_device(prog))
    B = P.attribute(rec)
    A = B.advise()
    Po = O.Program(prog)
    assert P.coverage() == O.coverage(Po)
    C, _ = O.count(Po.n_instr, rec)
    bl = Po.blame(C)
    for ri, root in enumerate(P.roots()):
        for opt in range(9):
            _hotspots_match(B.hotspots(ri, opt, 5), O.hotspots(Po, C, bl, int(root), opt, 5),
                            (which, int(root), opt))
    text = gpa.report(A, B, 5, 3)
    assert "single dependency coverage" in text and text.count("kernel (scope") == len(P.roots())
    A.close()
    B.close()
    P.close()
