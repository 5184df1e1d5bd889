#!/usr/bin/env python3
"""Throughput of the GPA hot path on one MI355X.

One step is one pass of the whole path over one profile of the large
single-kernel workload (60,000 instructions in 1,500 blocks, loop depth up to
5, 255 registers + 7 predicates + 16 barriers, 20M PC-sample records with
Zipf(1.2) PCs and a memory-dependency-heavy stall mix):

  load     gpa_load_program: validation, reaching definitions, def-use
           edges, CFG distances, static pruning and target scopes (Sec. 4);
  attribute gpa_attribute: sample histogram (Sec. 2.1) and blame with
           apportioning (Sec. 4.2, Eq. 1);
  advise   gpa_advise: scope roll-up, estimated speedups (Eqs. 2-5) and the
           ranked top-k, copied to the host.

Inputs are resident in HBM before timing starts.  Three copies of the sample
records (3 x 160 MB) are used in turn so that no step reads records another
step left in the 256 MB last-level cache.  `value` is records per second of
the whole step.  Kernel times come from the library's hipEvent pairs on the
streams the kernels run on; `roofline` is for the kernel family that takes
the most time per step, `roofline_hist` for the sample histogram, whose
traffic field comes from the rocprofv3 counter summary under profiles/ when
that summary was taken on the current source of the histogram kernels.  The CPU baseline is the oracle (test
infrastructure) run on the same workload on the host cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

HBM_PEAK_GBS = 8000.0
# 32-bit integer vector issue: 256 CUs x 64 lanes x 2.4 GHz, in Gops/s
ALU_PEAK_GOPS = 256 * 64 * 2.4e9 / 1e9
HIST_SOURCE = os.path.join(HERE, "paper_2009_04061_amd", "csrc", "hist.hip")
TRAFFIC_FILE = os.path.join(HERE, "profiles", "hist_large_traffic.json")


def _source_hash(path):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def _traffic(n_launches_ref=None):
    """HBM bytes per histogram pass from the committed counter summary, or
    None when it is absent or was taken on another version of the kernels."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_sha256_16") != _source_hash(HIST_SOURCE):
        return None
    return t.get("bytes_per_pass")


# the hot-set path (programs up to 2^17 instructions, the large workload) and
# the partition path beyond it
HIST_KERNELS = ("k_hot_select", "k_hot_pass", "k_hot_finish",
                "k_hsample", "k_hregions", "k_partition", "k_hplan", "k_count", "k_merge",
                "k_hoverflow")


def _counter_rows(d):
    """Rows of the rocprofv3 counter CSV files under directory d."""
    import csv
    import glob
    rows = []
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(f, newline="") as fh:
            rows.extend(csv.DictReader(fh))
    return rows


def summarize_traffic(fetch_dir, write_dir, copy_mb, out_path):
    """HBM bytes per histogram pass from two rocprofv3 --pmc runs (FETCH_SIZE,
    then WRITE_SIZE, KiB per dispatch), each scaled by what the same counter
    reads for the plain device copy of copy_mb MiB in the same run."""
    res = {}
    for counter, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        rows = [r for r in _counter_rows(d) if r.get("Counter_Name") == counter]
        if not rows:
            raise SystemExit(f"no {counter} rows under {d}")
        per_kernel = {}
        copy_vals = []
        for r in rows:
            name = r.get("Kernel_Name", "")
            v = float(r["Counter_Value"])
            if "copyBuffer" in name:
                copy_vals.append(v)
            for k in HIST_KERNELS:
                if ("gpa::" + k + "(") in name or ("gpa::" + k + "<") in name:
                    per_kernel.setdefault(k, []).append(v)
        if not copy_vals:
            raise SystemExit(f"no copy kernel in the {counter} run")
        copy_kib = max(copy_vals)   # the large calibration copy
        factor = (copy_mb * 1024.0) / copy_kib
        n_pass = max(len(v) for k, v in per_kernel.items()
                     if k in ("k_hot_pass", "k_partition", "k_count"))
        kib = sum(sum(v) for v in per_kernel.values()) / n_pass
        res[counter] = {"kib_per_pass_raw": kib, "copy_kib_raw": copy_kib,
                        "scale": factor, "bytes_per_pass": kib * 1024.0 * factor,
                        "per_kernel_kib_raw": {k: sum(v) / len(v) for k, v in per_kernel.items()}}
    out = {"kernel": "gpa_hist (sample histogram pass)",
           "workload": "large single kernel, 20M records",
           "source_sha256_16": _source_hash(HIST_SOURCE),
           "bytes_per_pass": res["FETCH_SIZE"]["bytes_per_pass"] +
                             res["WRITE_SIZE"]["bytes_per_pass"],
           "fetch": res["FETCH_SIZE"], "write": res["WRITE_SIZE"], "copy_mib": copy_mb}
    with open(out_path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


def cpu_baseline(prog, rec, seconds):
    """The oracle on the host: whole steps over the same workload until at
    least `seconds` of CPU work has been done (at least one step)."""
    from oracle import oracle
    oracle.build(force=False)
    times = []
    out = None
    t_all = time.perf_counter()
    while True:
        t0 = time.perf_counter()
        out = oracle.run_all(prog, rec, 5)
        times.append(time.perf_counter() - t0)
        if time.perf_counter() - t_all >= seconds:
            break
    med = statistics.median(times)
    n = len(rec)
    return {"value": n / med, "unit": "samples/s", "cores": 1, "kind": "oracle",
            "sample": f"the whole large workload ({n} records, {len(prog['op_class'])} "
                      f"instructions), {len(times)} single-thread oracle steps, median "
                      f"{med:.3f} s"}, out


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="minimum CPU time spent on the oracle baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true",
                    help="skip the comparison of one step with the oracle")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="after the timed steps, run a plain device copy of this many MiB "
                         "(calibrates the HBM byte counters of a profiling run)")
    ap.add_argument("--traffic-summary", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="no benchmark: turn two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) "
                         "of this script with --copy-mb into the traffic summary")
    args = ap.parse_args()

    if args.traffic_summary:
        summarize_traffic(args.traffic_summary[0], args.traffic_summary[1],
                          args.copy_mb or 512, TRAFFIC_FILE)
        return

    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the path has no multi-GPU code: one profile is processed by one GPU)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2009_04061_amd import gpa, synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    gpa.lib()   # fails loudly when the library is not built

    t0 = time.perf_counter()
    prog, rec = synth.workload_large(seed=1)
    gen_s = time.perf_counter() - t0
    n_rec = len(rec)
    n_instr = len(prog["op_class"])
    print(f"# workload generated in {gen_s:.1f} s: {n_instr} instructions, {n_rec} records",
          file=sys.stderr, flush=True)

    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    dprog = gpa.program_to_device(prog, dev)
    raw = np.ascontiguousarray(rec).view(np.uint8)
    copies = [torch.from_numpy(raw).to(dev) for _ in range(3)]
    torch.cuda.synchronize()

    def step(k):
        with torch.cuda.stream(stream):
            P = gpa.Program(dprog, stream=stream)
            B = P.attribute(copies[k % len(copies)], stream=stream)
            A = B.advise(stream=stream)
            top = A.topk(5)
        return P, B, A, top

    lat_adv = []
    for k in range(args.warmup):
        P, B, A, _ = step(k)
        A.close(); B.close(); P.close()
    torch.cuda.synchronize()

    gpa.timing_enable(True)
    gpa.timing_read(reset=True)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(args.steps):
        P, B, A, _ = step(k)
        A.close(); B.close(); P.close()
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    ph = gpa.timing_read(reset=True)
    gpa.timing_enable(False)

    # a program kept resident: attribute + advise per profile, and the advise
    # latency (host clock, from the call to the top-k on the host)
    P = gpa.Program(dprog, stream=stream)
    info = dict(P.info)
    lat_resident = []
    for k in range(args.steps):
        t_0 = time.perf_counter()
        B = P.attribute(copies[k % len(copies)], stream=stream)
        t_a = time.perf_counter()
        A = B.advise(stream=stream)
        A.topk(5)
        t_1 = time.perf_counter()
        lat_adv.append(t_1 - t_a)
        lat_resident.append(t_1 - t_0)
        A.close(); B.close()
    P.close()

    if args.copy_mb:
        a = torch.empty(args.copy_mb << 20, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        for _ in range(2):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    ms_step = 1e3 * t_total / args.steps
    value = n_rec * args.steps / t_total

    phase_ms = {name: (ms / c if c else None) for name, (ms, c) in ph.items()}
    rooflines = {}
    n_edges, n_scopes, n_blocks = info["n_edges"], info["n_scopes"], info["n_blocks"]
    n_succ = int(len(prog["succ"]))
    # walk-table relaxations: every source block against every sweep entry of
    # its function (one per predecessor edge, one per block without any),
    # once for shortest and once for longest walks
    fbb = np.asarray(prog["func_block_begin"], np.int64)
    n_pred = np.bincount(np.asarray(prog["succ"], np.int64), minlength=n_blocks)
    ent_per_block = np.maximum(n_pred, 1)
    ent_cum = np.concatenate([[0], np.cumsum(ent_per_block)])
    relax = 0
    for f in range(len(fbb) - 1):
        nb_f = int(fbb[f + 1] - fbb[f])
        relax += 2 * nb_f * int(ent_cum[fbb[f + 1]] - ent_cum[fbb[f]])
    # per-unit algorithmic work of each kernel family
    work = {
        "hist": ("hbm", 8.0 * n_rec + 96.0 * n_instr,
                 "gpa_hist: sample histogram (k_hot_select, k_hot_pass, k_hot_finish)"),
        "blame": ("hbm", 60.0 * n_edges + 288.0 * n_instr, "gpa_blame: k_blame_dst + k_blame_src"),
        "advise": ("hbm", 72.0 * n_scopes + 88.0 * n_instr + 8.0 * n_edges,
                   "gpa_estimate: contributions, scope sums, speedups, top-k"),
        "rd_search": ("hbm", 30.0 * n_instr, "gpa_dataflow: per-use backward searches"),
        "dfs": ("alu", float(n_blocks + n_succ), "CFG depth-first order (k_dfs)"),
        "dist": ("alu", float(relax) / 2,
                 "shortest-walk tables (k_dist_tables, block order): source blocks x sweep entries"),
        "dist_long": ("alu", float(relax) / 2,
                      "longest G' walk tables (k_dist_tables, DFS order): source blocks x sweep "
                      "entries"),
    }
    for name, (bound, amount, label) in work.items():
        t = phase_ms.get(name)
        if not t:
            continue
        if bound == "hbm":
            achieved, peak, unit = amount / (t * 1e-3) / 1e9, HBM_PEAK_GBS, "GB/s"
        else:
            achieved, peak, unit = amount / (t * 1e-3) / 1e9, ALU_PEAK_GOPS, "Gops/s"
        rooflines[name] = {"bound": bound, "kernel": label,
                           "achieved": float(f"{achieved:.6g}"),
                           "peak": peak, "unit": unit, "frac": float(f"{achieved / peak:.6g}"),
                           "traffic": _traffic() if name == "hist" else None,
                           "algorithmic": amount, "avg_ms": round(t, 5)}
    dominant = max(rooflines, key=lambda k: rooflines[k]["avg_ms"])
    roofline = dict(rooflines[dominant], name=dominant)
    roofline_hist = rooflines["hist"]

    checked = None
    base = None
    if not args.no_cpu_baseline:
        base, oracle_out = cpu_baseline(prog, rec, args.cpu_seconds)
        if not args.no_check:
            sys.path.insert(0, os.path.join(HERE, "tests"))
            from parity import compare, run_gpu   # noqa: E402
            g = run_gpu(prog, rec, device_inputs=True, k=5)
            compare(prog, g, oracle_out, k=5)
            checked = True

    a_sorted = sorted(lat_adv)
    p = lambda q: 1e3 * a_sorted[min(len(a_sorted) - 1, int(q * len(a_sorted)))]
    line = {
        "metric": "PC samples blamed/s, batched vs per-profile (oracle-exact); p99 advise latency",
        "value": round(value, 1), "unit": "samples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32+f64", "data": "synthetic",
        "config": {"workload": "large single kernel: 60k instructions, 1.5k blocks, loop depth "
                               "<= 5, 255 R + 7 P + 16 B, 20M records, Zipf 1.2, seed 1",
                   "records": n_rec, "instructions": n_instr, "path": "per-profile"},
        "phase_ms": {k: (round(v, 4) if v is not None else None) for k, v in phase_ms.items()},
        "advise_latency_ms": {"p50": round(p(0.5), 4), "p99": round(p(0.99), 4)},
        "samples_per_s_resident_program": round(n_rec / statistics.median(lat_resident), 1),
        "oracle_exact": checked,
        "roofline": roofline,
        "roofline_hist": roofline_hist,
        "cpu_baseline": base,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
