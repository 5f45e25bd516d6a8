"""GPU: the queued request server.  Every result must equal the same request
run alone on the per-set path (bit-identical: integer counts, one rounding),
whatever else is in flight, under a binding memory budget too."""
import sys
import time

import pytest

import causet_inputs as ci
import oracle

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def cs():
    import paper_1709_03013_amd as p
    return p


def oracle_result(d, N, seed):
    oc, _, _ = oracle.sprinkle(d, N, seed)
    h, R, sm = oracle.count_bits(oracle.link(d, oc), N, nbins=4) if N > 0 else ([0] * 4, 0, 0)
    return {"n": [int(x) for x in h[:4]], "R": R, "summ": sm,
            "S": oracle.bd_action(d, N, h[:4]) if N > 0 else oracle.bd_action(d, 0, [0] * 4), "status": 0}


def stored(name):
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "oracle_reference.json")) as f:
        return json.load(f)[name]


def alone(cs, ctx, d, N, seed):
    s = cs.cs_sprinkle(ctx, d, N, seed)
    try:
        cs.cs_link(ctx, s)
        n, R, sm = cs.cs_interval_abundances(ctx, s, 3, 0)
        return {"n": [int(x) for x in n], "R": R, "summ": sm, "S": cs.cs_bd_action(ctx, s), "status": 0}
    finally:
        cs.cs_set_free(s)


def run_all(cs, ctx, reqs, timeout_s=120):
    tickets = [cs.cs_queue_submit(ctx, d, N, seed) for d, N, seed in reqs]
    out = {}
    t0 = time.time()
    while len(out) < len(tickets):
        for t in tickets:
            if t in out:
                continue
            r = cs.cs_queue_poll(ctx, t)
            if r is not None:
                out[t] = r
        assert time.time() - t0 < timeout_s, "queue did not finish"
        time.sleep(0.001)
    return [out[t] for t in tickets]


MIX = [(2, 512, 1), (4, 700, 2), (2, 9000, 3), (4, 1500, 4), (2, 33, 5), (4, 0, 6), (2, 1, 7),
       (2, 20000, 8), (4, 5000, 9), (2, 2048, 10), (4, 12000, 11), (2, 777, 12), (4, 4096, 13),
       (2, 3000, 14), (2, 512, 1), (4, 700, 2)]


def test_results_in_the_mix_equal_alone(cs):
    say("case serve mix")
    ctx = cs.cs_create(0, 0, None)
    try:
        refs = [alone(cs, ctx, *r) for r in MIX]
        for req, ref in zip(MIX, refs):
            assert ref == oracle_result(*req), req
        cs.cs_queue_start(ctx, 4, 0)
        res = run_all(cs, ctx, MIX)
        for req, (r, tm), ref in zip(MIX, res, refs):
            assert r == ref, (req, r, ref)
            assert 0 <= tm[0] <= tm[2] and tm[1] >= 0
        # a second wave reuses resident matrices; results unchanged
        res2 = run_all(cs, ctx, MIX[::-1])
        assert [r for r, _ in res2] == refs[::-1]
        cs.cs_queue_drain(ctx)
    finally:
        cs.cs_destroy(ctx)


def test_binding_budget_admits_as_memory_frees(cs):
    """64 MiB budget: the 32768-element 2D matrix alone needs 128 MiB and is
    refused; everything else is admitted as slots and memory free up."""
    say("case serve budget")
    big = cs.cs_create(0, 0, None)
    ctx = cs.cs_create(0, 64 << 20, None)
    try:
        reqs = [(2, 8192, 20 + k) for k in range(6)] + [(4, 6000, 40 + k) for k in range(4)] + [(2, 32768, 99)]
        refs = [alone(cs, big, *r) for r in reqs[:-1]]
        cs.cs_queue_start(ctx, 3, 16 << 20)
        res = run_all(cs, ctx, reqs)
        for req, (r, _), ref in zip(reqs, res, refs):
            assert r == ref, req
        assert res[-1][0]["status"] == 2          # CS_ENOMEM
        assert cs.cs_bytes_in_use(ctx) <= 64 << 20
    finally:
        cs.cs_destroy(ctx)
        cs.cs_destroy(big)


def test_completion_order_interface(cs):
    """cs_queue_next hands out every finished request exactly once, in
    completion order, with the same results as polling by ticket; it times
    out with nothing pending."""
    say("case serve next")
    reqs = [(2, 3000 + 100 * k, 300 + k) for k in range(6)] + [(4, 2000, 400), (2, 512, 401)]
    ctx = cs.cs_create(0, 0, None)
    try:
        refs = {r: alone(cs, ctx, *r) for r in reqs}
        cs.cs_queue_start(ctx, 3, 0)
        assert cs.cs_queue_next(ctx, 0.0) is None
        tickets = {cs.cs_queue_submit(ctx, *r): r for r in reqs}
        got = {}
        t0 = time.time()
        while len(got) < len(reqs):
            r = cs.cs_queue_next(ctx, 1.0)
            assert time.time() - t0 < 120
            if r is None:
                continue
            t, res, tm = r
            assert t in tickets and t not in got
            assert res == refs[tickets[t]] and 0 <= tm[0] <= tm[2]
            got[t] = res
        assert cs.cs_queue_next(ctx, 0.05) is None
        # a ticket returned by cs_queue_next cannot be polled again
        with pytest.raises(cs.CsError):
            cs.cs_queue_poll(ctx, next(iter(tickets)))
    finally:
        cs.cs_destroy(ctx)


def test_queue_errors(cs):
    ctx = cs.cs_create(0, 0, None)
    try:
        with pytest.raises(cs.CsError):
            cs.cs_queue_submit(ctx, 2, 100, 1)      # not started
        cs.cs_queue_start(ctx, 2, 0)
        with pytest.raises(cs.CsError):
            cs.cs_queue_start(ctx, 2, 0)            # already running
        with pytest.raises(cs.CsError):
            cs.cs_queue_submit(ctx, 3, 100, 1)
        with pytest.raises(cs.CsError):
            cs.cs_queue_poll(ctx, 123456)
        t = cs.cs_queue_submit(ctx, 2, 300, 5)
        cs.cs_queue_drain(ctx)
        r, tm = cs.cs_queue_poll(ctx, t)
        assert r == alone(cs, ctx, 2, 300, 5)
    finally:
        cs.cs_destroy(ctx)


def test_request_plan_sample(cs):
    """A sample of the served workload (N log-uniform in [512, 32768]): every
    queued result equals the same request alone."""
    say("case serve plan sample")
    plan = ci.request_plan(60)
    reqs = [(d, N, seed) for _, d, N, seed in plan]
    ctx = cs.cs_create(0, 0, None)
    try:
        refs = [alone(cs, ctx, *r) for r in reqs]
        cs.cs_queue_start(ctx, 4, 0)
        res = run_all(cs, ctx, reqs)
        assert [r for r, _ in res] == refs
    finally:
        cs.cs_destroy(ctx)


def test_served_stream_sample_equals_oracle(cs):
    """Every 50th request of the 10,000-request served stream (200 requests,
    N up to 32768, both dimensions), queued together on 4 slots: each result
    equals the oracle's (stored by tests/golden/make_golden.py from oracle/
    only), bit for bit."""
    say("case serve vs oracle")
    sample = stored("served_sample")
    plan = ci.request_plan(sample["requests"])
    reqs = []
    for o in sample["results"]:
        _, d, N, seed = plan[o["q"]]
        assert (o["d"], o["N"], o["seed"]) == (d, N, seed), o["q"]
        reqs.append((d, N, seed))
    ctx = cs.cs_create(0, 0, None)
    try:
        cs.cs_queue_start(ctx, 4, 0)
        res = run_all(cs, ctx, reqs, timeout_s=300)
        for o, (r, _) in zip(sample["results"], res):
            assert r["status"] == 0, o["q"]
            assert r["n"] == o["n"] and r["R"] == o["R"] and r["summ"] == o["summ"], (o["q"], r, o)
            assert r["S"] == float.fromhex(o["S"]), (o["q"], r, o)
    finally:
        cs.cs_destroy(ctx)


def test_repeated_request_in_flight_waits_for_its_matrix(cs):
    """The same large request submitted several times back to back on four
    slots, twice over: a repeat must not read the resident matrix while the
    first copy is still building it.  Every result equals the oracle's."""
    say("case serve repeats in flight")
    reqs = [(2, 24000, 77)] * 4 + [(4, 16000, 78)] * 4 + [(2, 24000, 77), (4, 16000, 78)] * 2
    want = {r: oracle_result(*r) for r in set(reqs)}
    ctx = cs.cs_create(0, 0, None)
    try:
        cs.cs_queue_start(ctx, 4, 0)
        for rnd in range(2):
            res = run_all(cs, ctx, reqs)
            for req, (r, _) in zip(reqs, res):
                assert r == want[req], (rnd, req, r, want[req])
    finally:
        cs.cs_destroy(ctx)
