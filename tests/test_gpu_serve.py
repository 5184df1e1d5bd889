"""The serving loop (gpa_server_*): requests against resident programs,
admitted by device bytes, run in batches.  Each request's result must be bit
for bit the plain path's on the same records, alone or in the mix; a tiny
budget must queue requests (never more admitted bytes than the budget) and
refuse a request larger than the whole budget without blocking the rest."""
import time

import numpy as np
import pytest

from oracle import oracle as O
from paper_2009_04061_amd import synth as S
from parity import compare

pytestmark = pytest.mark.gpu


def _programs(k, seed=0):
    progs = []
    for i in range(k):
        progs.append(S.gen_program(seed=900 + seed * 100 + i, functions=[
            dict(n_instr=400 + 611 * i, n_blocks=10 + 7 * i, n_loops=3, max_depth=3, kind="kernel"),
            dict(n_instr=90, n_blocks=4, n_loops=1, max_depth=1, kind="device")],
            n_regs=48, n_preds=6, n_bars=6, inline_frac=0.05))
    return progs


def _result(P, B, A):
    C, tot = B.counts()
    return {"C": C, "totals": tot, "shares": B.shares(), "table": B.table(), "est": A.get(),
            "top": A.topk(16), "roots": P.roots(), "info": P.info, "rd": P.rd(), "edges": P.edges()}


def _same(a, b, where):
    for key in ("C", "totals", "shares"):
        assert np.array_equal(np.asarray(a[key]).view(np.uint8), np.asarray(b[key]).view(np.uint8)), \
            (where, key)
    for grp in ("table", "est", "top"):
        for key in a[grp]:
            assert np.array_equal(np.asarray(a[grp][key]).view(np.uint8),
                                  np.asarray(b[grp][key]).view(np.uint8)), (where, grp, key)


def _wait(server, tickets, timeout=120.0):
    done = {}
    t0 = time.time()
    while len(done) < len(tickets):
        for t in tickets:
            if t in done:
                continue
            r = server.poll(t, want_blame=True)
            if r is not None:
                done[t] = r
        assert time.time() - t0 < timeout, "requests did not finish"
        time.sleep(0.0005)
    return done


def test_each_result_is_the_same_alone_and_in_the_mix():
    import torch
    from paper_2009_04061_amd import gpa
    progs = _programs(6)
    P = [gpa.Program(gpa.program_to_device(p)) for p in progs]
    rng = np.random.default_rng(5)
    reqs = []
    for r in range(40):
        i = int(rng.integers(len(progs)))
        n = int(np.exp(rng.uniform(np.log(2_000), np.log(400_000))))
        rec = S.gen_samples(n, len(progs[i]["op_class"]), 1.1, S.stall_mix_small(), seed=1000 + r)
        # some requests come from device memory, the rest from the host
        src = torch.from_numpy(rec.view(np.uint8).copy()).cuda() if r % 4 == 0 else rec
        reqs.append((i, rec, src))
    sv = gpa.Server(64 << 30)
    tickets = [sv.submit(P[i], src) for i, _, src in reqs]
    done = _wait(sv, tickets)
    st = sv.stats()
    assert st["completed"] == len(reqs) and st["failed"] == 0
    print(f"server stats: {st}", flush=True)
    assert st["batches"] < len(reqs), "requests were never batched together"
    for t, (i, rec, src) in zip(tickets, reqs):
        A, B = done[t]
        got = _result(P[i], B, A)
        B1 = P[i].attribute(src)
        A1 = B1.advise()
        _same(got, _result(P[i], B1, A1), f"ticket {t}")
        A1.close(); B1.close(); A.close(); B.close()
    # and a few of them against the oracle
    for t, (i, rec, _) in list(zip(tickets, reqs))[:40:13]:
        B1 = P[i].attribute(rec)
        A1 = B1.advise()
        compare(progs[i], _result(P[i], B1, A1), O.run_all(progs[i], rec, k=16), k=16)
        A1.close(); B1.close()
    sv.close()


def test_wait_returns_each_finished_request_once():
    """gpa_server_wait hands out every finished ticket once, in finishing
    order; its results then poll at once; a ticket collected by a poll first
    is never handed out; an idle server's wait times out."""
    from paper_2009_04061_amd import gpa
    progs = _programs(3, seed=2)
    P = [gpa.Program(gpa.program_to_device(p)) for p in progs]
    sv = gpa.Server(64 << 30)
    assert sv.wait(0.001) is None
    recs = [S.gen_samples(20_000 + 3_000 * r, len(progs[r % 3]["op_class"]), 1.1,
                          S.stall_mix_small(), seed=3000 + r) for r in range(12)]
    tickets = [sv.submit(P[r % 3], rec) for r, rec in enumerate(recs)]
    seen = []
    while len(seen) < len(tickets):
        t = sv.wait(60.0)
        assert t is not None, "no request finished within a minute"
        seen.append(t)
        r = sv.poll(t)
        assert r is not None, "a waited-for ticket did not poll at once"
        r[0].close()
    assert sorted(seen) == sorted(tickets)
    assert sv.wait(0.001) is None
    # collected by polling, never handed out by a wait
    t = sv.submit(P[0], recs[0])
    done = _wait(sv, [t])
    done[t][0].close()
    done[t][1].close()
    assert sv.wait(0.01) is None
    sv.close()


def test_tiny_budget_queues_requests_and_refuses_oversize_ones():
    from paper_2009_04061_amd import gpa
    progs = _programs(3, seed=1)
    P = [gpa.Program(gpa.program_to_device(p)) for p in progs]
    budget = 96 << 20
    sv = gpa.Server(budget)
    # a request that alone needs more than the budget is refused at once
    big = S.gen_samples(6_000_000, len(progs[0]["op_class"]), 1.1, S.stall_mix_small(), seed=3)
    with pytest.raises(gpa.GpaError) as e:
        sv.submit(P[0], big)
    assert e.value.status == -2
    reqs = []
    for r in range(24):
        i = r % 3
        rec = S.gen_samples(900_000 + 1000 * r, len(progs[i]["op_class"]), 1.2,
                            S.stall_mix_memory_skewed(), seed=2000 + r)
        reqs.append((i, rec))
    tickets = [sv.submit(P[i], rec) for i, rec in reqs]
    done = _wait(sv, tickets)
    st = sv.stats()
    print(f"server stats: {st}", flush=True)
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert 0 < st["peak_reserved"] <= budget
    assert st["batches"] > 1, "the budget should have split the requests over batches"
    for t, (i, rec) in zip(tickets, reqs):
        A, B = done[t]
        B1 = P[i].attribute(rec)
        A1 = B1.advise()
        _same(_result(P[i], B, A), _result(P[i], B1, A1), f"ticket {t}")
        A1.close(); B1.close(); A.close(); B.close()
    # polled tickets are forgotten; unknown tickets are refused
    with pytest.raises(gpa.GpaError) as e:
        sv.poll(tickets[0])
    assert e.value.status == -1
    sv.close()


def test_server_free_with_unpolled_results_and_programs_freed_first():
    from paper_2009_04061_amd import gpa
    progs = _programs(2, seed=2)
    P = [gpa.Program(gpa.program_to_device(p)) for p in progs]
    sv = gpa.Server(8 << 30)
    for r in range(6):
        rec = S.gen_samples(50_000, len(progs[r % 2]["op_class"]), 1.1, S.stall_mix_small(),
                            seed=r)
        sv.submit(P[r % 2], rec)
    # the caller's program handles may go first: the server holds references
    for p in P:
        p.close()
    sv.close()     # waits for the requests and frees their results
