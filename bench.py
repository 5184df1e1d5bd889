#!/usr/bin/env python3
"""Throughput of the GPA hot path on one MI355X: batched vs per-profile.

The headline workload is the whole-application profile: 400 kernels with
2M instructions in all (log-normal sizes, device functions with their own
CFG, up to 12k function scopes) and 500M PC-sample records (4 GB) grouped by
kernel.  Programs are loaded once (the static analysis: reaching
definitions, edges, distances, target scopes; timed and reported apart), and
one step is the analysis of every kernel's records:

  batched      gpa_analyze_batch over all 400 kernels (gpa_attribute_batch and
               gpa_advise_batch in one call: each stage of the histogram,
               blamer and estimators one launch for the whole batch);
  per-profile  gpa_attribute + gpa_advise kernel by kernel (host loop).

`value` is records per second of the batched step, records resident in HBM
before timing starts.  Beside it, on the same GPU: the per-profile path on
the same records, the 1,024-profile batch (config 2) both ways, the large
single kernel (60,000 instructions, 20M records) on the per-profile path with
its load and step phases, and serving
(2,000 resident programs, requests of 50k-5M records on a 200 req/s Poisson
stream, admitted by a 64 GB budget): p50/p99 latency from submit to the
top-k on the host, against the per-request plain path.  Kernel times come
from the library's hipEvent pairs on the stream the phases run on;
`roofline` is for the phase that takes the most time per batched step.  The
CPU baseline is the oracle (test infrastructure) on a bounded sample of the
same kernels on the host.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import statistics
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

HBM_PEAK_GBS = 8000.0
# 32-bit integer vector issue: 256 CUs x 64 lanes x 2.4 GHz, in Gops/s
ALU_PEAK_GOPS = 256 * 64 * 2.4e9 / 1e9
HIST_SOURCE = os.path.join(HERE, "paper_2009_04061_amd", "csrc", "hist.hip")
TRAFFIC_FILE = os.path.join(HERE, "profiles", "hist_batch_wholeapp_traffic.json")
# the batched histogram's kernels: gpa::k_hot_*<..., true> (the last template
# argument selects the batched instantiation)
HIST_BATCH_RE = r"gpa::(k_hot_select|k_hot_pass|k_hot_finish)<(?:[^<>]*, )?true>"


def log(msg):
    print(f"# {msg}", file=sys.stderr, flush=True)


def _source_hash(path):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def _traffic():
    """HBM bytes per batched histogram from the committed counter summary,
    or None when it is absent or was taken on another version of the
    kernels."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_sha256_16") != _source_hash(HIST_SOURCE):
        return None
    return t.get("bytes_per_pass")


def _counter_rows(d):
    import csv
    import glob
    rows = []
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(f, newline="") as fh:
            rows.extend(csv.DictReader(fh))
    return rows


def summarize_traffic(fetch_dir, write_dir, copy_mb, out_path, steps):
    """HBM bytes per batched histogram from two rocprofv3 --pmc runs
    (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each scaled by what the
    same counter reads for the plain device copy of copy_mb MiB in the same
    run; `steps` histogram passes ran in each (warm-up included)."""
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
            m = re.search(HIST_BATCH_RE, name)
            if m:
                per_kernel.setdefault(m.group(1), []).append((int(r.get("Dispatch_Id", 0)), v))
        if not copy_vals:
            raise SystemExit(f"no copy kernel in the {counter} run")
        # the timed steps are the last `steps` dispatches of each kernel (the
        # warm-up and the autotuner's trial runs come before them)
        per_kernel = {k: [v for _, v in sorted(dv)[-steps:]] for k, dv in per_kernel.items()}
        copy_kib = max(copy_vals)
        factor = (copy_mb * 1024.0) / copy_kib
        kib = sum(sum(v) for v in per_kernel.values()) / steps
        res[counter] = {"kib_per_pass_raw": kib, "copy_kib_raw": copy_kib,
                        "scale": factor, "bytes_per_pass": kib * 1024.0 * factor,
                        "per_kernel_kib_raw": {k: sum(v) / steps for k, v in per_kernel.items()}}
    out = {"kernel": "gpa_hist batched (k_hot_select, k_hot_pass, k_hot_finish)",
           "workload": "whole application: 400 kernels, 2M instructions, 500M records",
           "source_sha256_16": _source_hash(HIST_SOURCE),
           "bytes_per_pass": res["FETCH_SIZE"]["bytes_per_pass"] +
                             res["WRITE_SIZE"]["bytes_per_pass"],
           "fetch": res["FETCH_SIZE"], "write": res["WRITE_SIZE"], "copy_mib": copy_mb}
    with open(out_path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


def summarize_kernels(trace_dir, out_path, steps, command):
    """A markdown table of the batched step's kernels from a rocprofv3
    --kernel-trace --stats run (CSV output) of this script: every kernel
    dispatched within the last `steps` batched steps of the headline workload
    (a step ends with the batched top-k's final kernel), with its average
    duration and its time per step."""
    import csv
    import glob
    rows = []
    for f in glob.glob(os.path.join(trace_dir, "**", "*kernel_trace.csv"), recursive=True):
        with open(f, newline="") as fh:
            rows.extend(csv.DictReader(fh))
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    ends = [int(r["End_Timestamp"]) for r in rows if "gpa::k_topk_final<true>" in r["Kernel_Name"]]
    if len(ends) < steps + 1:
        raise SystemExit("fewer batched steps in the trace than asked for")
    t0, t1 = ends[-steps - 1], ends[-1]
    per = {}
    for r in rows:
        b, e = int(r["Start_Timestamp"]), int(r["End_Timestamp"])
        if b <= t0 or e > t1:
            continue
        name = r["Kernel_Name"].split("(")[0]
        name = name[5:] if name.startswith("void ") else name
        per.setdefault(name, []).append((e - b) / 1e3)
    lines = ["# Batched step kernels: whole application (400 kernels, 500M records)", "",
             f"Command: `{command}`", "",
             f"Every kernel dispatched within the last {steps} batched steps (from the end "
             "of the step before them to the end of the last); durations from the "
             "kernel trace.", "",
             "| kernel | dispatches | avg µs | total per step µs |", "|---|---|---|---|"]
    tot = 0.0
    for name, d in sorted(per.items(), key=lambda kv: -sum(kv[1])):
        step_us = sum(d) / steps
        tot += step_us
        lines.append(f"| `{name}` | {len(d)} | {sum(d) / len(d):.1f} | {step_us:.1f} |")
    lines += ["", f"GPU time of the kernels per step: {tot / 1e3:.3f} ms; span of a step "
                  f"(wall, under the profiler): {(t1 - t0) / 1e6 / steps:.3f} ms."]
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def kernel_table(trace_dir, out_path, title, command):
    """A markdown table of every kernel in a rocprofv3 --kernel-trace --stats
    run (CSV output): dispatches, average and total duration, longest first."""
    import csv
    import glob
    rows = []
    for f in glob.glob(os.path.join(trace_dir, "**", "*kernel_trace.csv"), recursive=True):
        with open(f, newline="") as fh:
            rows.extend(csv.DictReader(fh))
    per = {}
    for r in rows:
        name = r.get("Kernel_Name", "").split("(")[0]
        if name.startswith("void "):
            name = name[5:]
        per.setdefault(name, []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    lines = [f"# {title}", "", f"Command: `{command}`", "",
             "| kernel | dispatches | avg µs | total µs |", "|---|---|---|---|"]
    for name, d in sorted(per.items(), key=lambda kv: -sum(kv[1])):
        lines.append(f"| `{name}` | {len(d)} | {sum(d) / len(d):.1f} | {sum(d):.1f} |")
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def _pct(values, q):
    v = sorted(values)
    return v[min(len(v) - 1, int(q * len(v)))]


# ------------------------------------------------------------------ pieces
def upload_records(torch, records, offsets, dev):
    """All profiles' records in one device buffer, each profile starting on a
    16-byte boundary; returns the per-profile byte views."""
    import numpy as np
    n = np.diff(offsets)
    starts = np.zeros(len(n) + 1, np.int64)
    starts[1:] = np.cumsum(n + (n & 1))
    buf = torch.empty(int(starts[-1]) * 8, dtype=torch.uint8, device=dev)
    raw = records.view(np.uint8)
    chunk = 64 << 20
    for k in range(len(n)):
        a, b = int(offsets[k]) * 8, int(offsets[k + 1]) * 8
        s = int(starts[k]) * 8
        for c in range(a, b, chunk):
            e = min(b, c + chunk)
            buf[s + c - a:s + e - a].copy_(torch.from_numpy(raw[c:e]), non_blocking=False)
    return buf, [buf[int(starts[k]) * 8:(int(starts[k]) + int(n[k])) * 8] for k in range(len(n))]


def load_programs(gpa, progs, dev, stream):
    t0 = time.perf_counter()
    P = [gpa.Program(gpa.program_to_device(p, dev), stream=stream) for p in progs]
    return P, time.perf_counter() - t0


def batched_step(gpa, inputs, stream):
    """gpa_analyze_batch (attribute + advise of every profile) with the top-k
    rows left on the device, then the batch's handles freed; `inputs` is the
    batch's argument arrays, marshalled once (gpa.BatchInputs)."""
    R = gpa.analyze_batch(inputs, stream=stream)
    R.close()


def per_profile_step(gpa, P, D, stream):
    for p, d in zip(P, D):
        b = p.attribute(d, stream=stream)
        a = b.advise(stream=stream)
        a.close()
        b.close()


def time_steps(torch, fn, steps):
    """Wall time per step; Python's cyclic garbage collector is paused over
    the timed steps (a full collection over the workload's host arrays would
    land inside one of them)."""
    import gc
    gc.collect()
    gc.disable()
    try:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps
    finally:
        gc.enable()


def run_batch_config(torch, gpa, cfg, steps, warmup, dev, stream, per_profile_steps=1):
    from paper_2009_04061_amd import synth
    t0 = time.perf_counter()
    progs, records, offsets = synth.gen_batch(cfg)
    log(f"config {cfg}: generated {len(progs)} profiles, {int(offsets[-1])} records in "
        f"{time.perf_counter() - t0:.1f} s")
    P, load_s = load_programs(gpa, progs, dev, stream)
    torch.cuda.synchronize()
    log(f"config {cfg}: loaded {len(P)} programs in {load_s:.2f} s")
    buf, D = upload_records(torch, records, offsets, dev)
    torch.cuda.synchronize()
    n_rec = int(offsets[-1])
    inputs = gpa.BatchInputs(P, D)
    for _ in range(warmup):
        batched_step(gpa, inputs, stream)
    # the timed steps run without the phase timers (their events are host
    # work between launches); as many steps again give the phase times
    t_batch = time_steps(torch, lambda: batched_step(gpa, inputs, stream), steps)
    gpa.timing_enable(True)
    gpa.timing_read(reset=True)
    time_steps(torch, lambda: batched_step(gpa, inputs, stream), steps)
    ph = gpa.timing_read(reset=True)
    gpa.timing_enable(False)
    log(f"config {cfg}: batched step {1e3 * t_batch:.2f} ms")
    per_profile_step(gpa, P, D, stream)   # warm-up of the plain path
    t_plain = time_steps(torch, lambda: per_profile_step(gpa, P, D, stream), per_profile_steps)
    log(f"config {cfg}: per-profile step {1e3 * t_plain:.2f} ms")
    info = {"instructions": int(sum(len(p["op_class"]) for p in progs)),
            "edges": int(sum(p.info["n_edges"] for p in P)),
            "scopes": int(sum(p.info["n_scopes"] for p in P)),
            "records": n_rec, "profiles": len(P)}
    out = {"records": n_rec, "t_batch": t_batch, "t_plain": t_plain, "load_s": load_s,
           "phases": {k: (ms / c if c else None) for k, (ms, c) in ph.items()}, "info": info}
    return out, progs, records, offsets, P, buf, D


def run_config1(torch, gpa, dev, stream, steps, loads=3):
    """The large single kernel (60,000 instructions in one function of 1,500
    blocks, 20M records) on the per-profile path: the program's load (static
    analysis) and one attribute + advise, each with the library's per-phase
    device times (load phases on the stream they run on; side-stream phases
    overlap the main one)."""
    import numpy as np
    from paper_2009_04061_amd import synth
    prog, rec = synth.workload_large(seed=1, n_samples=20_000_000)
    desc = gpa.program_to_device(prog, dev)
    gpa.Program(desc, stream=stream).close()          # warm-up load
    torch.cuda.synchronize()
    gpa.timing_enable(True)
    gpa.timing_read(reset=True)
    walls = []
    P = None
    for _ in range(loads):
        if P is not None:
            P.close()
        t0 = time.perf_counter()
        P = gpa.Program(desc, stream=stream)
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t0)
    lph = gpa.timing_read(reset=True)
    d = torch.from_numpy(np.ascontiguousarray(rec).view(np.uint8).copy()).to(dev)
    torch.cuda.synchronize()
    gpa.timing_enable(False)
    per_profile_step(gpa, [P], [d], stream)
    t_step = time_steps(torch, lambda: per_profile_step(gpa, [P], [d], stream), steps)
    gpa.timing_enable(True)
    gpa.timing_read(reset=True)
    time_steps(torch, lambda: per_profile_step(gpa, [P], [d], stream), steps)
    sph = gpa.timing_read(reset=True)
    gpa.timing_enable(False)
    info = P.info
    P.close()
    log(f"config 1: load {1e3 * min(walls):.2f} ms, step {1e3 * t_step:.3f} ms")
    per = lambda ph: {k: round(ms / c, 4) for k, (ms, c) in ph.items() if c}
    return {"workload": "large single kernel: 60,000 instructions in one function of 1,500 "
                        "blocks, loop depth <= 5, 20M records, Zipf 1.2, memory-skewed stall mix",
            "records": int(len(rec)), "instructions": int(info["n_instr"]),
            "edges": int(info["n_edges"]),
            "load_ms": round(1e3 * min(walls), 3), "load_phase_ms": per(lph),
            "step_ms": round(1e3 * t_step, 4), "step_phase_ms": per(sph),
            "samples_per_s": round(len(rec) / t_step, 1)}


def cpu_baseline(progs, records, offsets, seconds):
    """The oracle on the host over whole kernels of the workload, in order,
    until at least `seconds` of CPU work is done."""
    from oracle import oracle
    oracle.build(force=False)
    t_all = time.perf_counter()
    n_done = 0
    k = 0
    while k < len(progs):
        oracle.run_all(progs[k], records[offsets[k]:offsets[k + 1]], 5)
        n_done += int(offsets[k + 1] - offsets[k])
        k += 1
        if time.perf_counter() - t_all >= seconds:
            break
    el = time.perf_counter() - t_all
    return {"value": n_done / el, "unit": "samples/s", "cores": 1, "kind": "oracle",
            "sample": f"the first {k} of the {len(progs)} kernels of the whole-application "
                      f"workload ({n_done} records), single-thread oracle (count, sources, "
                      f"distances, blame, estimates, top-5 per kernel), {el:.1f} s"}


def serving(torch, gpa, dev, seconds, rate, budget, seed=4, n_programs=2000, pool=256):
    """Config 4: requests on a Poisson stream against resident programs."""
    import numpy as np
    from paper_2009_04061_amd import synth
    specs = synth.serving_specs(seed, n_programs)
    t0 = time.perf_counter()
    progs, _, _ = synth.gen_batch(4, specs=specs)
    log(f"serving: generated {len(progs)} programs in {time.perf_counter() - t0:.1f} s")
    P, load_s = load_programs(gpa, progs, dev, None)
    torch.cuda.synchronize()
    log(f"serving: loaded {len(P)} programs in {load_s:.2f} s")
    arrive, prog_of, n_of = synth.serving_requests(seed, n_programs, rate, seconds)
    # the request records: a pool of distinct (program, records) requests in
    # pinned host memory, drawn on the GPU, used in turn by the stream
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    reqs = []
    for r in range(min(pool, len(arrive))):
        p = int(prog_of[r])
        n = int(n_of[r])
        d = synth.gen_samples_device(n, len(progs[p]["op_class"]), specs[p]["zipf"],
                                     specs[p]["stall_mix"], g, device=dev)
        reqs.append((p, d.cpu().pin_memory()))
    torch.cuda.synchronize()
    log(f"serving: {len(reqs)} request buffers, {len(arrive)} arrivals over {seconds} s")

    def open_loop():
        sv = gpa.Server(budget)
        lat, pend = [], {}
        n_rec = 0
        t_start = time.perf_counter()
        i = 0
        while i < len(arrive) or pend:
            now = time.perf_counter() - t_start
            while i < len(arrive) and arrive[i] <= now:
                p, rec = reqs[i % len(reqs)]
                t = sv.submit(P[p], rec)
                pend[t] = (time.perf_counter(), rec.numel() // 8)
                i += 1
            # block until a request finishes or the next one arrives
            due = (arrive[i] - (time.perf_counter() - t_start)) if i < len(arrive) else 1.0
            if not pend:
                time.sleep(max(due, 0.0))
                continue
            t = sv.wait(max(due, 0.0))
            if t is None or t not in pend:
                continue
            A, _ = sv.poll(t)
            A.topk(5)
            t_sub, n = pend.pop(t)
            lat.append(time.perf_counter() - t_sub)
            n_rec += n
            A.close()
        el = time.perf_counter() - t_start
        st = sv.stats()
        sv.close()
        return lat, n_rec, el, st

    def saturated(count):
        sv = gpa.Server(budget)
        t0 = time.perf_counter()
        ts = [sv.submit(P[reqs[k % len(reqs)][0]], reqs[k % len(reqs)][1]) for k in range(count)]
        n_rec = sum(reqs[k % len(reqs)][1].numel() // 8 for k in range(count))
        left = set(ts)
        while left:
            t = sv.wait(60.0)
            if t is None or t not in left:
                continue
            A, _ = sv.poll(t)
            A.topk(5)
            A.close()
            left.discard(t)
        el = time.perf_counter() - t0
        st = sv.stats()
        sv.close()
        return n_rec / el, st

    def plain(count):
        lat = []
        n_rec = 0
        t0 = time.perf_counter()
        for k in range(count):
            p, rec = reqs[k % len(reqs)]
            t1 = time.perf_counter()
            B = P[p].attribute(rec)
            A = B.advise()
            A.topk(5)
            lat.append(time.perf_counter() - t1)
            n_rec += rec.numel() // 8
            A.close()
            B.close()
        return lat, n_rec / (time.perf_counter() - t0)

    saturated(min(64, len(reqs)))   # warm-up (autotuner buckets, code, pool)
    plain(8)
    lat, n_rec, el, st = open_loop()
    log(f"serving: open loop {len(lat)} requests, p50 {1e3 * _pct(lat, 0.5):.2f} ms, "
        f"p99 {1e3 * _pct(lat, 0.99):.2f} ms")
    sat_rate, sat_st = saturated(len(reqs))
    plat, prate = plain(len(reqs))
    log(f"serving: saturated {sat_rate:.3g} rec/s, plain {prate:.3g} rec/s")
    for p in P:
        p.close()
    return {
        "workload": f"{n_programs} resident programs (whole-application size law), Poisson "
                    f"{rate:g} req/s for {seconds:g} s, 50k-5M records log-uniform, budget "
                    f"{budget >> 30} GiB; request records from {len(reqs)} distinct "
                    f"(program, records) buffers in pinned host memory",
        "requests": len(lat), "programs_load_s": round(load_s, 3),
        "latency_ms": {"p50": round(1e3 * _pct(lat, 0.5), 3), "p99": round(1e3 * _pct(lat, 0.99), 3),
                       "max": round(1e3 * max(lat), 3)},
        "offered_samples_per_s": round(n_rec / el, 1),
        "saturated_samples_per_s": round(sat_rate, 1),
        "batches": st["batches"], "max_batch": st["max_batch"],
        "peak_reserved_bytes": st["peak_reserved"],
        "plain_path": {"latency_ms": {"p50": round(1e3 * _pct(plat, 0.5), 3),
                                      "p99": round(1e3 * _pct(plat, 0.99), 3)},
                       "samples_per_s": round(prate, 1)},
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="minimum CPU time spent on the oracle baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-config2", action="store_true", help="skip the 1,024-profile batch")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving run")
    ap.add_argument("--no-config1", action="store_true",
                    help="skip the large single-kernel profile (per-profile path)")
    ap.add_argument("--only-config1", action="store_true",
                    help="run only the large single-kernel profile and print its figures")
    ap.add_argument("--kernel-table", nargs=4, metavar=("TRACE_DIR", "OUT_MD", "TITLE", "COMMAND"),
                    help="write a table of every kernel of a rocprofv3 kernel trace "
                         "(COMMAND: the run that made the trace)")
    ap.add_argument("--serve-seconds", type=float, default=10.0)
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-budget-gib", type=int, default=64)
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="after the timed steps, run a plain device copy of this many MiB "
                         "(calibrates the HBM byte counters of a profiling run)")
    ap.add_argument("--traffic-summary", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="no benchmark: turn two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) "
                         "of this script with --copy-mb into the traffic summary")
    ap.add_argument("--kernel-summary", nargs=3, metavar=("TRACE_DIR", "OUT_MD", "COMMAND"),
                    help="no benchmark: turn a rocprofv3 --kernel-trace run (CSV) of this script "
                         "with --no-config2 into a markdown table of the batched step's kernels")
    args = ap.parse_args()

    if args.traffic_summary:
        summarize_traffic(args.traffic_summary[0], args.traffic_summary[1],
                          args.copy_mb or 512, TRAFFIC_FILE, args.steps)
        return
    if args.kernel_table:
        kernel_table(*args.kernel_table)
        return
    if args.kernel_summary:
        summarize_kernels(args.kernel_summary[0], args.kernel_summary[1], args.steps,
                          args.kernel_summary[2])
        return

    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(nothing in this path uses a second GPU; see the design notes for how it "
              "would shard)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2009_04061_amd import gpa

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    gpa.lib()   # fails loudly when the library is not built
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)

    if args.only_config1:
        print(json.dumps({"config1": run_config1(torch, gpa, dev, stream, args.steps)}), flush=True)
        return

    c3, progs, records, offsets, P, buf, D = run_batch_config(torch, gpa, 3, args.steps,
                                                              args.warmup, dev, stream)
    if args.copy_mb:
        a = torch.empty(args.copy_mb << 20, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        for _ in range(2):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    n_rec = c3["records"]
    info = c3["info"]
    ph = c3["phases"]
    for p in P:
        p.close()
    del buf, D, P

    # per-unit algorithmic work of each batched phase (design notes, sec. 7)
    work = {
        "hist": ("hbm", 8.0 * n_rec + 96.0 * info["instructions"],
                 "gpa_hist batched: k_hot_select, k_hot_pass, k_hot_finish"),
        "blame": ("hbm", 60.0 * info["edges"] + 288.0 * info["instructions"],
                  "gpa_blame batched: k_blame_dst + k_blame_src"),
        "advise": ("hbm", 72.0 * info["scopes"] + 88.0 * info["instructions"] + 8.0 * info["edges"],
                   "gpa_estimate batched: contributions, scope sums, speedups, top-k"),
    }
    rooflines = {}
    for name, (bound, amount, label) in work.items():
        t = ph.get(name)
        if not t:
            continue
        achieved = amount / (t * 1e-3) / 1e9
        rooflines[name] = {"bound": bound, "kernel": label, "achieved": float(f"{achieved:.6g}"),
                           "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": float(f"{achieved / HBM_PEAK_GBS:.6g}"),
                           "traffic": _traffic() if name == "hist" else None,
                           "algorithmic": amount, "avg_ms": round(t, 5)}
    dominant = max(rooflines, key=lambda k: rooflines[k]["avg_ms"])

    c2 = None
    if not args.no_config2:
        r2, *_ = run_batch_config(torch, gpa, 2, max(2, args.steps // 2), 1, dev, stream)
        c2 = {"workload": "1,024 kernel profiles: instructions log-normal (median 3k, 200-60k), "
                          "records log-normal (median 200k, 10k-10M), Dirichlet mixes, seed 2",
              "records": r2["records"], "instructions": r2["info"]["instructions"],
              "batched_samples_per_s": round(r2["records"] / r2["t_batch"], 1),
              "per_profile_samples_per_s": round(r2["records"] / r2["t_plain"], 1),
              "batched_ms_per_step": round(1e3 * r2["t_batch"], 3),
              "per_profile_ms_per_step": round(1e3 * r2["t_plain"], 3),
              "speedup": round(r2["t_plain"] / r2["t_batch"], 2),
              "programs_load_s": round(r2["load_s"], 3),
              "phase_ms": {k: round(v, 4) for k, v in r2["phases"].items() if v is not None}}

    c1 = None
    if not args.no_config1:
        c1 = run_config1(torch, gpa, dev, stream, args.steps)

    serve = None
    if not args.no_serving:
        serve = serving(torch, gpa, dev, args.serve_seconds, args.serve_rate,
                        args.serve_budget_gib << 30)

    base = None
    if not args.no_cpu_baseline:
        base = cpu_baseline(progs, records, offsets, args.cpu_seconds)

    value = n_rec / c3["t_batch"]
    line = {
        "metric": "PC samples blamed/s, batched vs per-profile (oracle-exact); p99 advise latency",
        "value": round(value, 1), "unit": "samples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(1e3 * c3["t_batch"], 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32+f64",
        "data": "synthetic",
        "config": {"workload": "whole application: 400 kernels, 2M instructions (log-normal "
                               "sizes), <= 12k function scopes, 500M records (4 GB) grouped by "
                               "kernel, Zipf 1.1, Dirichlet mixes, seed 3",
                   "records": n_rec, "instructions": info["instructions"],
                   "edges": info["edges"], "scopes": info["scopes"],
                   "profiles": info["profiles"], "path": "batched, programs resident"},
        "per_profile_samples_per_s": round(n_rec / c3["t_plain"], 1),
        "per_profile_ms_per_step": round(1e3 * c3["t_plain"], 3),
        "batched_vs_per_profile": round(c3["t_plain"] / c3["t_batch"], 2),
        "programs_load_s": round(c3["load_s"], 3),
        "samples_per_s_including_load": round(n_rec / (c3["t_batch"] + c3["load_s"]), 1),
        "phase_ms": {k: (round(v, 4) if v is not None else None) for k, v in ph.items()
                     if v is not None},
        "roofline": dict(rooflines[dominant], name=dominant),
        "roofline_hist": rooflines.get("hist"),
        "config2": c2,
        "config1": c1,
        "serving": serve,
        "cpu_baseline": base,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
