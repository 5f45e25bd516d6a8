"""Write the stored oracle results used by the parity tests.

Calls only ``oracle/`` (and the shared input generators).  Every value in
``oracle_reference.json`` comes from this script; rerun it after a change to
the oracle's arithmetic and justify the change in the commit message.

    python tests/golden/make_golden.py            # small and medium workloads
    python tests/golden/make_golden.py --large    # also the 2D N=131072 workload
    python tests/golden/make_golden.py --plans    # the 512-set ensemble and a
                                                  # sample of the served stream
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import causet_inputs as ci  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(HERE, "oracle_reference.json")

CASES = {
    # name: (d, N, seed, full histogram?)
    "2d_1024": (2, 1024, 1, True),
    "4d_2048": (4, 2048, 14, True),
    "2d_5000": (2, 5000, 21, False),
    "4d_16384": (4, 16384, 2, False),
    "2d_131072": (2, 131072, 3, False),
}


def run_case(d, N, seed, full):
    t0 = time.time()
    coords, _, drawn = oracle.sprinkle(d, N, seed)
    bits = oracle.link(d, coords)
    nb = max(N - 1, 4) if full else 4
    hist, R, summ = oracle.count_bits(bits, N, nbins=nb)
    S = oracle.bd_action(d, N, hist[:4])
    rec = {
        "d": d, "N": N, "seed": seed, "candidates": drawn,
        "n": [int(x) for x in hist[:4]], "R": R, "summ": summ,
        "S": S.hex(), "S_float": S,
        "bitset_sha256": hashlib.sha256(bits.tobytes()).hexdigest(),
        "coords_sha256": hashlib.sha256(np.ascontiguousarray(coords).tobytes()).hexdigest(),
        "three_chains": oracle.three_chains(bits, N),
        "seconds": round(time.time() - t0, 2),
    }
    if full:
        last = int(np.nonzero(hist)[0].max()) + 1 if hist.any() else 1
        rec["hist_full"] = [int(x) for x in hist[:last]]
    return rec


# The served stream's stored sample: every SERVED_STEP-th request of the
# 10,000-request plan.
SERVED_REQUESTS = 10000
SERVED_STEP = 50


def plan_record(d, N, seed):
    """Abundances, R, sum of interior counts and the action of one sprinkled
    set, as the plan tests compare them."""
    coords, _, _ = oracle.sprinkle(d, N, seed)
    bits = oracle.link(d, coords)
    hist, R, summ = oracle.count_bits(bits, N, nbins=4)
    S = oracle.bd_action(d, N, hist[:4])
    return {"d": d, "N": N, "seed": seed, "n": [int(x) for x in hist[:4]], "R": R,
            "summ": summ, "S": S.hex()}


def run_plans(data):
    t0 = time.time()
    data["ensemble_512"] = [plan_record(d, N, seed) for d, N, seed in ci.ensemble_plan(512)]
    print("ensemble_512: %.1f s" % (time.time() - t0), flush=True)
    plan = ci.request_plan(SERVED_REQUESTS)
    sample = []
    t0 = time.time()
    for q in range(0, SERVED_REQUESTS, SERVED_STEP):
        _, d, N, seed = plan[q]
        rec = plan_record(d, N, seed)
        rec["q"] = q
        sample.append(rec)
        print("served q=%d d=%d N=%d: %.1f s" % (q, d, N, time.time() - t0), flush=True)
    data["served_sample"] = {"requests": SERVED_REQUESTS, "step": SERVED_STEP, "results": sample}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--large", action="store_true")
    ap.add_argument("--only", default=None)
    ap.add_argument("--plans", action="store_true")
    a = ap.parse_args()
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    if a.plans:
        run_plans(data)
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        return
    for name, (d, N, seed, full) in CASES.items():
        if a.only and name != a.only:
            continue
        if N > 20000 and not a.large:
            continue
        print("case", name, flush=True)
        data[name] = run_case(d, N, seed, full)
        print(json.dumps({k: v for k, v in data[name].items() if k != "hist_full"}), flush=True)
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
