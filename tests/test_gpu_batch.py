"""GPU: the batched ensemble path (one hipGraph replay per call) against the
per-set path and the oracle.  Results are integers and one rounding, so
"the same" means bit-identical."""
import sys

import numpy as np
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


@pytest.fixture(scope="module")
def ctx(cs):
    c = cs.cs_create(0, 0, None)
    yield c
    cs.cs_destroy(c)


def per_set(cs, ctx, d, N, seed):
    s = cs.cs_sprinkle(ctx, d, N, seed)
    try:
        cs.cs_link(ctx, s)
        n, R, sm = cs.cs_interval_abundances(ctx, s, 3, 0)
        S = cs.cs_bd_action(ctx, s) if N >= 0 else 0.0
        return {"n": [int(x) for x in n], "R": R, "summ": sm, "S": S, "status": 0}
    finally:
        cs.cs_set_free(s)


MIXED = [(2, 0, 5), (2, 1, 6), (4, 2, 7), (2, 63, 8), (4, 65, 9), (2, 300, 10), (4, 777, 11),
         (2, 2048, 12), (4, 2049, 13), (2, 4096, 14), (4, 3000, 15), (2, 9000, 16), (4, 8200, 17),
         (2, 16384, 18)]


def test_batch_call_reused_arrays_match_cs_batch_run(cs, ctx):
    # BatchCall marshals once and calls the library repeatedly: every call
    # overwrites the same result array with the same results
    say("case batch call reuse")
    plan = MIXED[5:10]
    ref = cs.cs_batch_run(ctx, plan)
    call = cs.BatchCall(plan)
    for _ in range(3):
        call.run(ctx)
        assert call.results() == ref


def test_batch_mixed_sizes_match_per_set_and_oracle(cs, ctx):
    say("case batch mixed")
    res = cs.cs_batch_run(ctx, MIXED)
    for (d, N, seed), r in zip(MIXED, res):
        ref = per_set(cs, ctx, d, N, seed)
        assert r == ref, (d, N, seed, r, ref)
        if N <= 3000:
            oc, _, _ = oracle.sprinkle(d, N, seed)
            h, R, sm = oracle.count_bits(oracle.link(d, oc), N, nbins=4)
            assert r["n"] == [int(x) for x in h] and r["R"] == R and r["summ"] == sm
            assert r["S"] == oracle.bd_action(d, N, h)


def test_batch_tuner_keeps_results_and_reports_its_choices(cs):
    """A fresh context tunes the batch on its first call: every (d, N-bucket)
    group is counted by the popcount kernel and by both matrix-core tile
    shapes (the tuner itself fails the batch if any candidate's counts
    differ), and the chosen kinds cover every set.  A second context that
    already knows the groups reuses the choices.  Results equal the per-set
    path both times."""
    say("case batch tuner")
    plan = MIXED[:12]
    c1 = cs.cs_create(0, 0, None)
    try:
        refs = [per_set(cs, c1, *p) for p in plan]
        res = cs.cs_batch_run(c1, plan)
        assert res == refs
        info = cs.cs_batch_last_info(c1)
        counted = sum(1 for d, N, _ in plan if N >= 2)
        assert info["sets_pop"] + info["sets_mfma256"] + info["sets_mfma128"] == counted, info
        assert info["count_ms_untuned"] > 0 and info["count_ms_tuned"] > 0, info
        for k in ("pop", "mfma256", "mfma128"):
            assert (info["grid_" + k] > 0) == (info["sets_" + k] > 0), info
        # same context, new shape containing the same groups: no new tuning of
        # those groups, same results as alone
        plan2 = plan[::-1]
        assert cs.cs_batch_run(c1, plan2) == refs[::-1]
    finally:
        cs.cs_destroy(c1)


def test_ensemble_means_match_2d_expectations(cs, ctx):
    """8192 2D diamonds of N = 256 in one batch: the sample means of
    N_0..N_3 equal the exact expectations over random 2D orders (a rational
    closed form, pinned against all orders of N <= 7 in the oracle tests),
    and the mean action equals 2 (Eq. 4 in expectation), each within five
    standard errors of the sample."""
    from test_oracle_count import expected_abundance_2d
    N, sets = 256, 8192
    say("case ensemble means N=%d sets=%d" % (N, sets))
    res = cs.cs_batch_run(ctx, [(2, N, 700000 + k) for k in range(sets)])
    n = np.array([r["n"] for r in res], dtype=np.float64)
    S = np.array([r["S"] for r in res])
    se = n.std(axis=0, ddof=1) / np.sqrt(sets)
    exp = np.array([float(expected_abundance_2d(N, k)) for k in range(4)])
    assert np.all(np.abs(n.mean(axis=0) - exp) < 5 * se), (n.mean(axis=0), exp, se)
    assert abs(S.mean() - 2.0) < 5 * S.std(ddof=1) / np.sqrt(sets), (S.mean(), S.std())


def test_graph_replays_with_eager_work_between(cs, ctx):
    say("case batch replays")
    plan = [(2, 500, 1), (4, 700, 2), (2, 1200, 3), (4, 9000, 4)]
    first = cs.cs_batch_run(ctx, plan)
    refs = [per_set(cs, ctx, *p) for p in plan]
    assert first == refs
    for rep in range(4):
        # eager work on the same context between replays
        per_set(cs, ctx, 2, 333, 100 + rep)
        again = cs.cs_batch_run(ctx, plan)
        assert again == refs, rep
    # same shape, new seeds: the replay must pick them up
    plan2 = [(d, N, seed + 1000) for d, N, seed in plan]
    res2 = cs.cs_batch_run(ctx, plan2)
    assert res2 == [per_set(cs, ctx, *p) for p in plan2]
    assert res2 != refs


def test_invalid_requests_get_their_own_status(cs, ctx):
    plan = [(2, 100, 1), (3, 100, 2), (4, -5, 3), (2, 10**6, 4), (4, 100, 5)]
    res = cs.cs_batch_run(ctx, plan)
    assert [r["status"] for r in res] == [0, 1, 1, 1, 0]
    assert res[0] == per_set(cs, ctx, 2, 100, 1)
    assert res[4] == per_set(cs, ctx, 4, 100, 5)


def stored(name):
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "oracle_reference.json")) as f:
        return json.load(f)[name]


def test_ensemble_workload_512_sets(cs, ctx):
    """The 512-set ensemble (N uniform in [256, 4096], d in {2, 4}): every set
    equals the oracle (stored by tests/golden/make_golden.py from oracle/
    only) and its own per-set run."""
    say("case ensemble 512")
    plan = ci.ensemble_plan(512)
    ref = stored("ensemble_512")
    res = cs.cs_batch_run(ctx, plan)
    for k, ((d, N, seed), r, o) in enumerate(zip(plan, res, ref)):
        assert (o["d"], o["N"], o["seed"]) == (d, N, seed), k
        assert r["n"] == o["n"] and r["R"] == o["R"] and r["summ"] == o["summ"], (k, r, o)
        assert r["S"] == float.fromhex(o["S"]) and r["status"] == 0, (k, r, o)
    for k in range(0, 512, 1):
        d, N, seed = plan[k]
        assert res[k] == per_set(cs, ctx, d, N, seed), k
    # and a few computed by the oracle here, not read back
    for k in (0, 1, 2, 3, 100, 511):
        d, N, seed = plan[k]
        oc, _, _ = oracle.sprinkle(d, N, seed)
        h, R, sm = oracle.count_bits(oracle.link(d, oc), N, nbins=4)
        assert res[k]["n"] == [int(x) for x in h] and res[k]["R"] == R and res[k]["summ"] == sm


def test_batch_budget_error(cs):
    c = cs.cs_create(0, 1 << 20, None)
    try:
        with pytest.raises(cs.CsError) as e:
            cs.cs_batch_run(c, [(2, 4096, 1)] * 8)
        assert e.value.status == 2
    finally:
        cs.cs_destroy(c)
