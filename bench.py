"""Benchmark: interval pairs/s and BD actions/s on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--path P] [--no-cpu] [--no-batch]
                    [--no-serve] [--no-pop] [--no-span] [--no-desitter]

One step = the whole hot path on the 2D flat causal diamond with N = 131072
elements (seed 3): sprinkle + time sort, link (2 GiB packed matrix), interval
counting (abundances N_0..N_3, R, sum of interior counts) and the BD action,
all through the C ABI.  Inputs are synthetic (the paper's workloads are
sprinklings too).  ``value`` = related pairs whose interval size was computed,
per second of the whole step.

Also reported on the same line:
  * roofline: the counting kernel (the dominant one), timed with HIP events
    on the library's stream over the timed region;
  * cpu_baseline: the CPU oracle's counting rate on a bounded row sample of
    the same set, on this host's cores;
  * kernels: the link kernel's HBM rate, and the popcount kernel on the same
    matrix (once) with its integer-ALU fraction;
  * other_configs: the 2D N=1024 and 4D N=16384 single-set workloads;
  * ensemble: 512 sets (N uniform in [256, 4096], d in {2, 4}) as BD
    actions/s, batched (one cs_batch_run) vs per-set (a loop of cs_* calls);
  * desitter: ten (1+1) de Sitter slabs of 2^15 elements (eta0 = 0.5), the
    smeared action at eps = 2^-6 against 4 pi tan(eta0);
  * served: 10,000 queued requests (N log-uniform in [512, 32768]) with
    Poisson arrivals at 0.7x the saturated rate, p50/p99 latency and
    actions/s, under a 32 GiB and a 1 GiB budget.

Protocol: W warm-up steps (default 3), then K timed steps (default 5);
ms_per_step is their mean, count/link kernel times are also given as min and
median.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD = dict(d=2, N=131072, seed=3)
PEAK = {
    "int8_mfma_tops": 5.0e15,      # dense int8 MFMA, ops/s
    "fp4_mfma_flops": 10.1e15,     # dense fp4 MFMA, flop/s
    "alu_int32_ops": 256 * 64 * 2.4e9,  # 256 CU x 64 lanes x 2.4 GHz, 32-bit VALU ops/s
    "hbm_bytes": 8.0e12,
}


# HBM traffic per launch of a count kernel on this workload: rocprofv3 --pmc
# FETCH_SIZE and WRITE_SIZE (KiB per dispatch), each divided by what the same
# counter reads per byte of a plain device-to-device copy.  Keyed by the
# SHA-256 of the kernel's source files when the counters were taken: after
# any change to them the figure no longer describes the kernel and is
# reported as null.
TRAFFIC = {
    # FETCH_SIZE 50336831 KiB / 0.5 (the counter reads 0.5 KiB per KiB of a
    # plain copy) + WRITE_SIZE 93312 KiB / 1.0, per launch on this workload
    "k_count_mfma_lds<fp4>": {"sources": "32e4b5e1ad42d22b", "bytes": 103375151281},
    "k_sat_tile": {"sources": "8152c5cd84815ecb", "bytes": 40494117034},
    "k_count_pop": {"sources": "a7be8e83898c0202", "bytes": 2541606105923},
}
KERNEL_SOURCES = {
    "k_count_mfma_lds<int8>": ["k_count_mfma.hip", "cs_device.h", "cs_internal.h"],
    "k_count_mfma_lds<fp4>": ["k_count_mfma.hip", "cs_device.h", "cs_internal.h"],
    "k_count_mfma<int8>": ["k_count_mfma.hip", "cs_device.h", "cs_internal.h"],
    "k_count_mfma<fp4>": ["k_count_mfma.hip", "cs_device.h", "cs_internal.h"],
    "k_count_pop": ["k_count_pop.hip", "cs_device.h", "cs_internal.h"],
    "k_sat_tile": ["k_count_sat.hip", "cs_device.h", "cs_internal.h"],
}


def sources_digest(kernel: str) -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_1709_03013_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_bytes(kernel: str):
    t = TRAFFIC.get(kernel)
    if t is None or t["sources"] != sources_digest(kernel):
        return None
    return t["bytes"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def span_words(bits: np.ndarray, N: int) -> int:
    """W_alg = sum over related pairs i<j of the number of 64-bit words that
    hold columns i+1..j-1 (the words Alg. 5 ANDs and counts)."""
    log("span_words: counting the span of every related pair of N=%d on the host" % N)
    W = bits.shape[1]
    tot = 0
    rowblk = 1024
    wi = np.arange(W, dtype=np.int64)
    for lo in range(0, N, rowblk):
        hi = min(lo + rowblk, N)
        blk = bits[lo:hi]
        i = np.arange(lo, hi, dtype=np.int64)[:, None]
        # keep columns j > i only
        first = (i + 1) >> 6
        keep = np.where(wi[None, :] > (i >> 6), np.uint64(0xFFFFFFFFFFFFFFFF), np.uint64(0))
        same = wi[None, :] == (i >> 6)
        shift = ((i & 63) + 1).astype(np.uint64)
        above = np.where(shift >= 64, np.uint64(0), (~np.uint64(0)) << np.minimum(shift, 63).astype(np.uint64))
        keep = np.where(same, above, keep)
        x = blk & keep
        cnt = np.bitwise_count(x).astype(np.int64)
        # a related j in word w spans words first..(j-1)>>6: (w - first + 1), minus one if j%64 == 0
        b0 = (x & np.uint64(1)).astype(np.int64)
        tot += int((cnt * (wi[None, :] - first + 1)).sum() - b0.sum())
    # adjacent related pairs (j = i+1) span no word; the formula gave them one
    i = np.arange(N - 1, dtype=np.int64)
    j = i + 1
    adj = (bits[i, j >> 6] >> (j & 63).astype(np.uint64)) & np.uint64(1)
    tot -= int(adj[(j & 63) != 0].sum())
    return tot


def mfma_roofline(N: int, t: float, fp4: bool) -> dict:
    """Matrix-core count: 2*C(N,3) operations (one multiply and one add per
    triple i < k < j) in t seconds against the dense peak of its operand type."""
    ops = 2.0 * math.comb(N, 3)
    # the library's kernel shape (CS_MFMA_VARIANT, default 12: LDS-staged, 2x4 waves,
    # 4 stages, weighted spreading, XCD-grouped tile order, unscaled fp4 encoding)
    lds = int(os.environ.get("CS_MFMA_VARIANT", "12")) >= 2
    kernel = ("k_count_mfma_lds" if lds else "k_count_mfma") + ("<fp4>" if fp4 else "<int8>")
    r = {"bound": "mfma", "achieved": ops / t / 1e12,
         "peak": (PEAK["fp4_mfma_flops"] if fp4 else PEAK["int8_mfma_tops"]) / 1e12,
         "unit": "TFLOP/s", "kernel": kernel,
         "work": "2*C(N,3) operations (multiply + add per triple i<k<j), %s operands"
                 % ("fp4 e2m1 0/1" if fp4 else "int8 0/1 (an int8 operation counted as a flop)")}
    r["frac"] = r["achieved"] / r["peak"]
    r["traffic"] = traffic_bytes(kernel)
    r["sources"] = sources_digest(kernel)
    return r


def pop_roofline(walg, t: float) -> dict:
    """Popcount count: 4 int32 VALU operations (2 AND, 2 bit counts) per
    64-bit word of every related pair's span."""
    ops = 4.0 * walg if walg else float("nan")
    r = {"bound": "alu", "achieved": ops / t / 1e12, "peak": PEAK["alu_int32_ops"] / 1e12,
         "unit": "TOP/s", "kernel": "k_count_pop",
         "work": "4 int32 ops per 64-bit word of the span of every related pair (W_alg=%s)" % walg}
    r["frac"] = r["achieved"] / r["peak"]
    r["traffic"] = traffic_bytes("k_count_pop")
    r["sources"] = sources_digest("k_count_pop")
    return r


def sat_dense_words(N: int, C: int) -> int:
    """64-bit words the saturating count's dense step reads per pair, summed
    over its 64x64 tiles: every word of [bi, bj] when bj - bi + 1 <= C + 2,
    else the C-word chunk."""
    nb = (N + 63) // 64
    tot = 0
    for g in range(nb):           # g = bj - bi, nb - g tiles
        span = g + 1
        tot += (nb - g) * (span if span <= C + 2 else C)
    return tot


def local_figures(cs, ctx, s, stream, ev, n_exact, R_exact, t_exact) -> dict:
    """The saturating count (N_0..N_3 and R only) on the bench matrix: time
    (HIP events on the library's stream, 1 warm-up + 3 timed calls) and the
    VALU bound of its dense step (4 int32 ops per pair and word, 4096 pairs
    per tile); the rest of the kernel (pairs continued past the window) has
    no data-independent work count."""
    C = int(os.environ.get("CS_SAT_CHUNK", "8"))
    cs.cs_local_abundances(ctx, s)
    ms = []
    for _ in range(3):
        ev[1].record(stream)
        n, R, q = cs.cs_local_abundances(ctx, s)
        ev[2].record(stream)
        ev[2].synchronize()
        ms.append(ev[1].elapsed_time(ev[2]))
    t = float(np.mean(ms)) / 1000.0
    N = WORKLOAD["N"]
    ops = 4.0 * 4096 * sat_dense_words(N, C)
    r = {"bound": "alu", "achieved": ops / t / 1e12, "peak": PEAK["alu_int32_ops"] / 1e12,
         "unit": "TOP/s", "kernel": "k_sat_tile",
         "work": "dense step only: 4 int32 ops per pair and word, 4096 pairs per 64x64 tile, "
                 "C=%d words per tile (all of [bi, bj] when it spans <= C+2 words)" % C}
    r["frac"] = r["achieved"] / r["peak"]
    r["count_ms"] = {"mean": t * 1000.0, "min": float(np.min(ms)), "median": float(np.median(ms))}
    r["pairs_per_s"] = R / t
    r["speedup_vs_exact"] = t_exact / t
    r["equals_exact"] = (list(n) == list(n_exact) and R == R_exact)
    r["continued_from_hbm"] = q
    r["traffic"] = traffic_bytes("k_sat_tile")
    r["sources"] = sources_digest("k_sat_tile")
    log("local (saturating) count on the same set: %.1f ms" % (t * 1000.0))
    return r


def link_figures(N: int, W: int, link_ms) -> dict:
    """Link kernel: N*W*8 bytes of matrix written (coordinate reads are
    N*16 bytes and negligible) per launch."""
    t = float(np.mean(link_ms)) / 1000.0
    byt = N * W * 8
    return {"bound": "hbm", "achieved": byt / t / 1e9, "peak": PEAK["hbm_bytes"] / 1e9,
            "unit": "GB/s", "frac": byt / t / PEAK["hbm_bytes"], "bytes": byt,
            "link_ms": {"mean": t * 1000.0, "min": float(np.min(link_ms)),
                        "median": float(np.median(link_ms))}}


def run_step(cs, ctx, ev, stream, path):
    """One pass of the hot path; ev[0..2] bracket link and count on the
    library's stream."""
    d, N, seed = WORKLOAD["d"], WORKLOAD["N"], WORKLOAD["seed"]
    s = cs.cs_sprinkle(ctx, d, N, seed)
    ev[0].record(stream)
    cs.cs_link(ctx, s)
    ev[1].record(stream)
    n, R, sm = cs.cs_interval_abundances(ctx, s, 3, path)
    ev[2].record(stream)
    S = cs.cs_bd_action(ctx, s)
    return s, n, R, sm, S


def cpu_baseline(budget_s: float = 12.0):
    import oracle
    d, N, seed = WORKLOAD["d"], WORKLOAD["N"], WORKLOAD["seed"]
    t0 = time.time()
    coords, _, _ = oracle.sprinkle(d, N, seed)
    bits = oracle.link(d, coords)
    t_link = time.time() - t0
    nthreads = oracle.num_threads()
    # evenly spaced 64-row blocks until the time budget is used
    starts = [int(x) for x in np.linspace(0, N - 64, 64)]
    order = [starts[k] for k in np.random.default_rng(0).permutation(len(starts))]
    pairs = 0
    rows = 0
    t_count = 0.0
    log("cpu_baseline: oracle link of N=%d done in %.1f s on %d threads" % (N, t_link, nthreads))
    for lo in order:
        t1 = time.time()
        _, R, _ = oracle.count_bits(bits, N, nbins=4, rows=(lo, lo + 64))
        t_count += time.time() - t1
        pairs += R
        rows += 64
        log("cpu_baseline: rows %d..%d, %.1f s so far" % (lo, lo + 63, t_count))
        if t_count > budget_s:
            break
    cpu = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            cpu = next(l.split(":", 1)[1].strip() for l in f if l.startswith("model name"))
    except (OSError, StopIteration):
        pass
    return {
        "value": pairs / t_count, "unit": "interval pairs/s", "cores": nthreads, "kind": "oracle",
        "cpu": cpu, "affinity": len(os.sched_getaffinity(0)),
        "sample": "%d rows (64-row blocks evenly spread over the N=131072 2D set, seed 3): interval "
                  "counts of all %d related pairs (i,j) with i in the sample, %.1f s; the oracle's "
                  "full link (%.1f s) not included" % (rows, pairs, t_count, t_link),
    }


def ensemble(cs, ctx, nsets=512):
    import causet_inputs as ci
    plan = ci.ensemble_plan(nsets)
    out = {}
    try:
        cs.cs_batch_run(ctx, plan)  # warm-up (graph capture, tuning)
        log("ensemble: warm-up batch done")
        t0 = time.time()
        res = cs.cs_batch_run(ctx, plan)
        tb = time.time() - t0
        log("ensemble: batched %d sets in %.3f s" % (nsets, tb))
        out["batched_actions_per_s"] = nsets / tb
        out["batched_s"] = tb
    except cs.CsError as e:
        out["batched_error"] = str(e)
        res = None
    t0 = time.time()
    per = []
    for (d, N, seed) in plan:
        s = cs.cs_sprinkle(ctx, d, N, seed)
        cs.cs_link(ctx, s)
        n, R, sm = cs.cs_interval_abundances(ctx, s, 3, 0)
        per.append((list(map(int, n)), R, sm, cs.cs_bd_action(ctx, s)))
        cs.cs_set_free(s)
    tp = time.time() - t0
    log("ensemble: per-set loop %d sets in %.3f s" % (nsets, tp))
    out["per_set_actions_per_s"] = nsets / tp
    out["per_set_s"] = tp
    if res is not None:
        out["batched_equals_per_set"] = all(
            r["n"] == p[0] and r["R"] == p[1] and r["summ"] == p[2] and r["S"] == p[3]
            for r, p in zip(res, per))
    out["sets"] = nsets
    return out


def small_configs(cs, ctx, stream, ev):
    """The other two single-set workloads: 2D N=1024 (seed 1) and 4D N=16384
    (seed 2).  Whole step and count call timed, 3 warm-ups, 5 timed."""
    out = {}
    for name, d, N, seed in (("2d_1024", 2, 1024, 1), ("4d_16384", 4, 16384, 2)):
        steps, counts = [], []
        for k in range(8):
            t0 = time.perf_counter()
            s = cs.cs_sprinkle(ctx, d, N, seed)
            cs.cs_link(ctx, s)
            ev[1].record(stream)
            n, R, sm = cs.cs_interval_abundances(ctx, s, 3, 0)
            ev[2].record(stream)
            S = cs.cs_bd_action(ctx, s)
            ev[2].synchronize()
            if k >= 3:
                steps.append((time.perf_counter() - t0) * 1e3)
                counts.append(ev[1].elapsed_time(ev[2]))
            path = cs.cs_set_count_path(s)
            cs.cs_set_free(s)
        out[name] = {"N": N, "d": d, "related_pairs": R, "abundances": [int(x) for x in n], "action": S,
                     "count_path": {1: "pop", 2: "mfma_int8", 3: "mfma_fp4"}[path],
                     "ms_per_step": float(np.mean(steps)), "count_ms": float(np.mean(counts)),
                     "pairs_per_s": R / (float(np.mean(steps)) / 1e3)}
        log("%s: step %.3f ms, count %.3f ms (%s)" % (name, out[name]["ms_per_step"], out[name]["count_ms"],
                                                     out[name]["count_path"]))
    return out


def desitter(cs, ctx, N=32768, graphs=10, eta0=0.5, eps=2.0**-6,
             sweep=((1024, 10), (4096, 10), (16384, 10), (65536, 10), (131072, 10))):
    """The paper's de Sitter experiment (Sec. 6.1): (1+1) de Sitter slabs at
    eta0, the smeared action with eps against the continuum value
    4 pi tan(eta0).  Ten graphs at N (timed), then the convergence sweep over
    (N, graphs) from 2^10 to 2^17 elements."""
    def run(n, g, seed0):
        S = []
        t0 = time.time()
        for k in range(g):
            s = cs.cs_sprinkle_desitter(ctx, n, seed0 + k, eta0)
            cs.cs_link(ctx, s)
            S.append(cs.cs_smeared_action(ctx, s, eps))
            cs.cs_set_free(s)
        t = time.time() - t0
        return S, t

    S, t = run(N, graphs, 1000)
    log("desitter: %d graphs of N=%d in %.2f s" % (graphs, N, t))
    by_n = []
    for n, g in sweep:
        Sn, tn = run(n, g, 2000)
        by_n.append({"N": n, "graphs": g, "seeds": "2000..%d" % (2000 + g - 1),
                     "S_eps_mean": float(np.mean(Sn)),
                     "S_eps_sd": float(np.std(Sn, ddof=1)) if g > 1 else None,
                     "graphs_per_s": g / tn})
        log("desitter sweep: N=%d, %d graphs, S_eps %.3f, %.2f s" % (n, g, np.mean(Sn), tn))
    return {"N": N, "graphs": graphs, "eta0": eta0, "eps": eps, "seeds": "1000..%d" % (1000 + graphs - 1),
            "S_eps_mean": float(np.mean(S)), "S_eps_sd": float(np.std(S, ddof=1)),
            "S_EH": 4 * math.pi * math.tan(eta0), "graphs_per_s": graphs / t, "by_N": by_n}


def served(cs, nreq=10000, slots=4, budget_gib=32.0, load=0.7):
    """Served stream: requests with Poisson arrivals (N log-uniform in
    [512, 32768], d in {2, 4}).  The saturated rate is measured first on a
    burst of the first 1500 requests; the timed run offers all requests at
    `load` times that rate.  Half the budget may hold resident matrices."""
    import causet_inputs as ci
    plan = ci.request_plan(nreq)
    ctx = cs.cs_create(0, int(budget_gib * 2**30), None)
    try:
        cs.cs_queue_start(ctx, slots, int(budget_gib * 2**30 / 2))

        def drive(reqs, arrivals):
            t0 = time.perf_counter()
            pending = {}
            lat = []
            k = 0
            done = 0
            while done < len(reqs):
                now = time.perf_counter() - t0
                while k < len(reqs) and (arrivals is None or arrivals[k] <= now):
                    d, N, seed = reqs[k]
                    pending[cs.cs_queue_submit(ctx, d, N, seed)] = k
                    k += 1
                for t in list(pending):
                    r = cs.cs_queue_poll(ctx, t)
                    if r is not None:
                        res, tm = r
                        assert res["status"] == 0
                        lat.append(tm[2])
                        del pending[t]
                        done += 1
                        if done % 1000 == 0:
                            log("served (%g GiB): %d/%d done, %.1f s" % (budget_gib, done, len(reqs),
                                                                        time.perf_counter() - t0))
                if k < len(reqs) and arrivals is not None:
                    time.sleep(max(0.0, min(0.0005, arrivals[k] - (time.perf_counter() - t0))))
            return time.perf_counter() - t0, np.array(lat)

        reqs = [(d, N, seed) for _, d, N, seed in plan]
        cal_n = min(1500, nreq)
        t_cal, _ = drive(reqs[:cal_n], None)
        sat = cal_n / t_cal
        log("served (%g GiB): saturated %.0f actions/s on a burst of %d" % (budget_gib, sat, cal_n))
        rate = load * sat
        gaps = np.array([a for a, *_ in plan])
        gaps = gaps / gaps[-1] * (nreq / rate)  # rescale the Poisson arrivals to `rate`
        t_run, lat = drive(reqs, gaps)
        return {"requests": nreq, "slots": slots, "hbm_budget_gib": budget_gib,
                "saturated_actions_per_s": sat, "offered_rate_per_s": rate,
                "actions_per_s": nreq / t_run, "p50_ms": float(np.percentile(lat, 50) * 1e3),
                "p99_ms": float(np.percentile(lat, 99) * 1e3), "wall_s": t_run}
    finally:
        cs.cs_destroy(ctx)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--path", type=int, default=0, help="0 auto, 1 popcount, 2 MFMA")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-span", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-pop", action="store_true", help="skip the one popcount-path count")
    ap.add_argument("--no-desitter", action="store_true")
    ap.add_argument("--no-local", action="store_true", help="skip the saturating-count leg")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only copy BYTES between two device buffers 3 times (calibrates HBM counters)")
    ap.add_argument("--serve-requests", type=int, default=10000)
    a = ap.parse_args()
    if a.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(its sharding is a design, not code); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    if a.copy_probe:
        # a plain device-to-device copy of known size: what FETCH_SIZE and
        # WRITE_SIZE read for it calibrates those counters for the count kernel
        n = a.copy_probe // 8
        src = torch.arange(n, dtype=torch.int64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": n * 8, "copies": 3}))
        return

    import paper_1709_03013_amd as cs

    torch.cuda.init()
    stream = torch.cuda.Stream(device=0)
    ctx = cs.cs_create(0, 0, stream.cuda_stream)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]

    for _ in range(a.warmup):
        s, *_ = run_step(cs, ctx, ev, stream, a.path)
        cs.cs_set_free(s)
    torch.cuda.synchronize()
    log("warm-up done (%d steps)" % a.warmup)
    count_ms, link_ms, step_ms = [], [], []
    t0 = time.perf_counter()
    for k in range(a.steps):
        ts = time.perf_counter()
        s, n, R, sm, S = run_step(cs, ctx, ev, stream, a.path)
        ev[2].synchronize()
        step_ms.append((time.perf_counter() - ts) * 1000.0)
        link_ms.append(ev[0].elapsed_time(ev[1]))
        count_ms.append(ev[1].elapsed_time(ev[2]))
        if k + 1 < a.steps:
            cs.cs_set_free(s)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1000.0 / a.steps
    log("step %.1f ms, count %s ms, link %s ms" % (ms_step, ["%.1f" % x for x in count_ms],
                                                  ["%.2f" % x for x in link_ms]))

    N = WORKLOAD["N"]
    W = cs.cs_row_words(N)
    path_used = cs.cs_set_count_path(s)
    t_count = float(np.mean(count_ms)) / 1000.0
    if path_used in (2, 3):
        roof = mfma_roofline(N, t_count, path_used == 3)
    else:
        walg = None if a.no_span else span_words(cs.cs_get_bitset(ctx, s), N)
        roof = pop_roofline(walg, t_count)
    roof["count_ms"] = {"mean": float(np.mean(count_ms)), "min": float(np.min(count_ms)),
                        "median": float(np.median(count_ms))}
    kernels = {"link": link_figures(N, W, link_ms)}
    if not a.no_pop and path_used != 1:
        # the popcount kernel on the same matrix, once, for its ALU fraction
        ev[1].record(stream)
        n1, R1, sm1 = cs.cs_interval_abundances(ctx, s, 3, 1)
        ev[2].record(stream)
        ev[2].synchronize()
        t_pop = ev[1].elapsed_time(ev[2]) / 1000.0
        walg = None if a.no_span else span_words(cs.cs_get_bitset(ctx, s), N)
        kernels["pop"] = pop_roofline(walg, t_pop)
        kernels["pop"]["count_ms"] = t_pop * 1000.0
        kernels["pop"]["equals_mfma"] = (list(n1) == list(n) and R1 == R and sm1 == sm)
        log("popcount path on the same set: %.1f ms" % (t_pop * 1000.0))
    if not a.no_local:
        kernels["local"] = local_figures(cs, ctx, s, stream, ev, n, R, t_count)
    cs.cs_set_free(s)

    small = small_configs(cs, ctx, stream, ev)
    ens = None if a.no_batch else ensemble(cs, ctx)
    dsx = None if a.no_desitter else desitter(cs, ctx)
    srv = None
    if not a.no_serve:
        srv = {"unbound_32gib": served(cs, a.serve_requests, budget_gib=32.0),
               "bound_1gib": served(cs, a.serve_requests, budget_gib=1.0)}
    cpu = None if a.no_cpu else cpu_baseline()
    cs.cs_destroy(ctx)

    rec = {
        "metric": "interval pairs/s & BD actions/s: batched vs per-set, 2D N=2^17",
        "value": R / (ms_step / 1000.0),
        "unit": "interval pairs/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {1: "u32", 2: "i8", 3: "fp4"}[path_used], "data": "synthetic",
        "config": {"workload": "2D flat causal diamond, N=131072, seed 3 (sprinkle+sort+link+count+action)",
                   "N": N, "d": 2, "related_pairs": R, "abundances": [int(x) for x in n],
                   "action": S, "count_path": {1: "pop", 2: "mfma_int8", 3: "mfma_fp4"}[path_used]},
        "roofline": roof,
        "kernels": kernels,
        "other_configs": small,
        "cpu_baseline": cpu,
        "ensemble": ens,
        "desitter": dsx,
        "served": srv,
    }
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
