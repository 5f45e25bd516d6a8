"""GPU parity: the HIP path, called through the C ABI, against the oracle.

Integer outputs (coordinates as bit patterns, matrix words, abundances, R,
sum of interior counts) must match bit-exactly; the FP64 action must match
to 1e-12 relative (it is in fact bit-identical: one rounding of an exact
integer bracket on both sides).  Sizes span several 64-row tiles and ragged
tails; the full-size workloads are checked against stored oracle results.
"""
import json
import os
import sys

import numpy as np
import pytest

import causet_inputs as ci
import oracle

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden", "oracle_reference.json")
REL_TOL = 1e-12


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


def action_close(a, b):
    return abs(a - b) <= REL_TOL * max(abs(b), 1.0)


def gpu_set(cs, ctx, d, N, seed):
    s = cs.cs_sprinkle(ctx, d, N, seed)
    cs.cs_link(ctx, s)
    return s


# ------------------------------------------------------------- sprinkle/link
@pytest.mark.parametrize("d,N,seed", [(2, 0, 1), (2, 1, 1), (2, 2, 5), (2, 63, 2), (2, 64, 3),
                                      (2, 65, 4), (2, 1024, 1), (2, 2047, 6), (2, 2048, 7),
                                      (2, 2049, 8), (2, 5000, 21), (4, 1, 3), (4, 2, 9),
                                      (4, 129, 10), (4, 2048, 14), (4, 3001, 11)])
def test_sprinkle_and_link_match_oracle(cs, ctx, d, N, seed):
    say("case sprinkle+link d=%d N=%d seed=%d" % (d, N, seed))
    s = gpu_set(cs, ctx, d, N, seed)
    try:
        assert cs.cs_set_manifold(s) == (cs.CS_MANIFOLD_DIAMOND, d)
        coords, orig = cs.cs_get_coords(ctx, s)
        oc, oo, _ = oracle.sprinkle(d, N, seed)
        assert np.array_equal(coords.view(np.uint64), oc.view(np.uint64))
        assert np.array_equal(orig, oo)
        bits = cs.cs_get_bitset(ctx, s)
        assert np.array_equal(bits, oracle.link(d, oc))
    finally:
        cs.cs_set_free(s)


# ------------------------------------------------------------------- counts
@pytest.mark.parametrize("path", [1, 2, 3])
@pytest.mark.parametrize("d,N,seed", [(2, 2, 1), (2, 3, 2), (2, 64, 3), (2, 65, 4), (2, 200, 5),
                                      (2, 255, 16), (2, 256, 17), (2, 257, 18), (2, 1024, 1),
                                      (2, 1500, 12), (2, 2304, 19), (4, 64, 6), (4, 300, 7),
                                      (4, 2048, 14), (4, 2500, 15), (2, 4096, 21), (4, 4097, 20)])
def test_counts_match_oracle(cs, ctx, d, N, seed, path):
    say("case count d=%d N=%d seed=%d path=%d" % (d, N, seed, path))
    s = gpu_set(cs, ctx, d, N, seed)
    try:
        n, R, sm = cs.cs_interval_abundances(ctx, s, 3, path)
        oc, _, _ = oracle.sprinkle(d, N, seed)
        h, oR, osm = oracle.count_bits(oracle.link(d, oc), N, nbins=4)
        assert list(n) == list(h) and R == oR and sm == osm
        S = cs.cs_bd_action(ctx, s)
        So = oracle.bd_action(d, N, h)
        assert action_close(S, So) and S == So
    finally:
        cs.cs_set_free(s)


@pytest.mark.parametrize("d,N,seed", [(2, 2049, 8), (2, 4100, 9), (4, 3001, 11), (4, 300, 12),
                                      (2, 511, 13), (2, 512, 14), (2, 513, 15), (4, 1025, 16),
                                      (2, 1537, 17), (4, 64, 18), (2, 65, 19), (2, 3, 20)])
def test_link_ragged_sizes_match_oracle(cs, ctx, d, N, seed):
    """The link writes the oracle's matrix byte for byte at sizes on and
    around the 64-label blocks and the 512-label tiles, 2D and 4D."""
    say("case link d=%d N=%d" % (d, N))
    s = gpu_set(cs, ctx, d, N, seed)
    try:
        oc, _, _ = oracle.sprinkle(d, N, seed)
        assert np.array_equal(cs.cs_get_bitset(ctx, s), oracle.link(d, oc))
    finally:
        cs.cs_set_free(s)


@pytest.mark.parametrize("d,N,seed", [(2, 700, 7), (4, 1500, 8), (2, 3000, 2)])
def test_mfma_paths_every_histogram_length_match_oracle(cs, ctx, d, N, seed):
    """Both matrix-core operand types, N_0..N_3, 41 bins and the full
    histogram: bins, R and the sum of interior counts equal the oracle's.
    (2D N=3000 with 41 bins is where a removed 2x2-wave int8 form once
    returned a wrong sum of interior counts with correct bins.)"""
    say("case mfma histograms d=%d N=%d" % (d, N))
    s = gpu_set(cs, ctx, d, N, seed)
    try:
        oc, _, _ = oracle.sprinkle(d, N, seed)
        ob = oracle.link(d, oc)
        for k in (3, 40, N - 2):
            h, oR, osm = oracle.count_bits(ob, N, nbins=k + 1)
            for path in (2, 3):
                n, R, sm = cs.cs_interval_abundances(ctx, s, k, path)
                assert np.array_equal(n, h) and R == oR and sm == osm, (path, k)
    finally:
        cs.cs_set_free(s)


@pytest.mark.parametrize("path", [1, 2, 3])
@pytest.mark.parametrize("kmax", [4, 17, 200])
@pytest.mark.parametrize("d,N,seed", [(2, 700, 31), (4, 1100, 32)])
def test_full_histogram_matches_oracle(cs, ctx, d, N, seed, kmax, path):
    say("case fullhist d=%d N=%d kmax=%d path=%d" % (d, N, kmax, path))
    s = gpu_set(cs, ctx, d, N, seed)
    try:
        n, R, sm = cs.cs_interval_abundances(ctx, s, kmax, path)
        oc, _, _ = oracle.sprinkle(d, N, seed)
        h, oR, osm = oracle.count_bits(oracle.link(d, oc), N, nbins=kmax + 1)
        assert np.array_equal(n, h) and R == oR and sm == osm
    finally:
        cs.cs_set_free(s)


@pytest.mark.parametrize("path", [1, 2, 3])
def test_row_block_stats_match_oracle(cs, ctx, path):
    d, N, seed = 2, 1300, 41
    say("case rowblocks N=%d path=%d" % (N, path))
    s = gpu_set(cs, ctx, d, N, seed)
    try:
        blocks = cs.cs_interval_abundances_rows(ctx, s, 5, path)
        oc, _, _ = oracle.sprinkle(d, N, seed)
        bits = oracle.link(d, oc)
        for b in range(blocks.shape[0]):
            lo, hi = b * 256, min(b * 256 + 256, N)
            h, R, sm = oracle.count_bits(bits, N, nbins=6, rows=(lo, hi))
            assert list(blocks[b, :6]) == list(h) and blocks[b, 6] == R and blocks[b, 7] == sm
    finally:
        cs.cs_set_free(s)


# ------------------------------------------------------------ injected orders
def injected_cases():
    return [
        ("chain", ci.chain_order(130)),
        ("chain1", ci.chain_order(1)),
        ("antichain", ci.antichain_order(77)),
        ("layers2", ci.layered_order([40, 90])),
        ("layers3", ci.layered_order([30, 50, 70])),
        ("dag", ci.random_dag_order(500, 0.01, 3)),
        ("union", ci.disjoint_union(ci.chain_order(64), ci.layered_order([5, 9, 3]),
                                    ci.random_dag_order(100, 0.05, 4))),
    ]


@pytest.mark.parametrize("path", [1, 2, 3])
@pytest.mark.parametrize("name,order", injected_cases(), ids=[c[0] for c in injected_cases()])
def test_injected_orders(cs, ctx, name, order, path):
    say("case injected %s path=%d" % (name, path))
    N = order.shape[0]
    bits = ci.pack_symmetric(order)
    s = cs.cs_set_from_bitset(ctx, 2, N, bits)
    try:
        n, R, sm = cs.cs_interval_abundances(ctx, s, 3, path)
        h, oR, osm = oracle.count_bits(bits, N, nbins=4)
        assert list(n) == list(h) and R == oR and sm == osm
        if name == "chain":
            assert cs.cs_bd_action(ctx, s) == 2.0 * N
        if name == "antichain":
            assert cs.cs_bd_action(ctx, s) == 2.0 * N
    finally:
        cs.cs_set_free(s)


def test_injected_chain_coordinates_action(cs, ctx):
    for d in (2, 4):
        N = 300
        s = cs.cs_set_from_coords(ctx, d, ci.chain_coords(d, N))
        cs.cs_link(ctx, s)
        S = cs.cs_bd_action(ctx, s)
        assert S == (2.0 * N if d == 2 else oracle.bd_action(4, N, [N - 1, N - 2, N - 3, N - 4]))
        cs.cs_set_free(s)
        s = cs.cs_set_from_coords(ctx, d, ci.antichain_coords(d, N))
        cs.cs_link(ctx, s)
        n, R, _ = cs.cs_interval_abundances(ctx, s, 3, 0)
        assert R == 0 and not n.any()
        cs.cs_set_free(s)


def test_validation_rejects_bad_matrices(cs, ctx):
    bits = ci.pack_symmetric(ci.chain_order(70))
    bad = bits.copy()
    bad[3, 0] ^= 1 << 10          # breaks symmetry
    with pytest.raises(cs.CsError):
        cs.cs_set_from_bitset(ctx, 2, 70, bad)
    bad = bits.copy()
    bad[5, 0] |= 1 << 5           # diagonal
    with pytest.raises(cs.CsError):
        cs.cs_set_from_bitset(ctx, 2, 70, bad)
    bad = bits.copy()
    bad[5, 1] |= 1 << 20          # padding column 84 >= N
    with pytest.raises(cs.CsError):
        cs.cs_set_from_bitset(ctx, 2, 70, bad)


# ------------------------------------------------------------- device tier
@pytest.mark.parametrize("d", [2, 4])
def test_device_pointer_tier_with_torch(cs, d):
    """cs_link_dev and cs_count_dev on torch-owned memory (row stride wider
    than W; 2D with its link tables in a caller workspace): the oracle's
    matrix, zero words past W, and its counts."""
    import torch
    say("case device tier d=%d" % d)
    N, seed = 1000, 51
    oc, _, _ = oracle.sprinkle(d, N, seed)
    W = cs.cs_row_words(N)
    coords = torch.from_numpy(oc).to("cuda:0")
    bits = torch.full((N, W + 4), -1, dtype=torch.int64, device="cuda:0")   # wider stride
    stats = torch.zeros(6, dtype=torch.int64, device="cuda:0")
    work = torch.zeros(cs.cs_count_workspace_bytes(N, 3) // 8, dtype=torch.int64, device="cuda:0")
    lw = cs.cs_link_workspace_bytes(d, N)
    assert lw == (2112 * ((N + 63) // 64) if d == 2 else 0)
    lwork = torch.full((max(lw, 8) // 8,), -1, dtype=torch.int64, device="cuda:0")
    stream = torch.cuda.current_stream().cuda_stream
    cs.cs_link_dev(d, N, coords.data_ptr(), bits.data_ptr(), W + 4, lwork.data_ptr() if lw else None, lw, stream)
    cs.cs_count_dev(bits.data_ptr(), N, W + 4, 3, stats.data_ptr(), work.data_ptr(), 0, stream)
    torch.cuda.synchronize()
    ob = oracle.link(d, oc)
    got = bits.cpu().numpy().view(np.uint64)
    assert np.array_equal(got[:, :W], ob) and not got[:, W:].any()
    h, R, sm = oracle.count_bits(ob, N, nbins=4)
    st = stats.cpu().numpy().view(np.uint64)
    assert list(st[:4]) == list(h) and st[4] == R and st[5] == sm


@pytest.mark.parametrize("path", [1, 2, 3])
@pytest.mark.parametrize("kmax", [3, 50])
def test_device_pointer_tier_paths(cs, path, kmax):
    """cs_count_dev on a torch-owned matrix (stride wider than W) with each
    count path and a histogram past bin 3: the oracle's bins, R and sum."""
    import torch
    d, N, seed = 2, 3000, 52
    say("case device tier path=%d kmax=%d" % (path, kmax))
    oc, _, _ = oracle.sprinkle(d, N, seed)
    ob = oracle.link(d, oc)
    W = cs.cs_row_words(N)
    bits = torch.zeros((N, W + 12), dtype=torch.int64)
    bits[:, :W] = torch.from_numpy(ob.view(np.int64))
    bits = bits.to("cuda:0")
    stats = torch.zeros(kmax + 3, dtype=torch.int64, device="cuda:0")
    work = torch.zeros(cs.cs_count_workspace_bytes(N, kmax) // 8, dtype=torch.int64, device="cuda:0")
    stream = torch.cuda.current_stream().cuda_stream
    cs.cs_count_dev(bits.data_ptr(), N, W + 12, kmax, stats.data_ptr(), work.data_ptr(), path, stream)
    torch.cuda.synchronize()
    h, R, sm = oracle.count_bits(ob, N, nbins=kmax + 1)
    st = stats.cpu().numpy().view(np.uint64)
    assert np.array_equal(st[:kmax + 1], h) and st[kmax + 1] == R and st[kmax + 2] == sm


def test_histogram_longer_than_the_set(cs, ctx):
    """kmax beyond N - 2: the bins past the largest possible interval are 0."""
    N, seed, kmax = 60, 53, 200
    s = gpu_set(cs, ctx, 2, N, seed)
    try:
        oc, _, _ = oracle.sprinkle(2, N, seed)
        h, R, sm = oracle.count_bits(oracle.link(2, oc), N, nbins=N - 1)
        for path in (1, 2, 3):
            n, gR, gsm = cs.cs_interval_abundances(ctx, s, kmax, path)
            assert np.array_equal(n[:N - 1], h) and not n[N - 1:].any() and gR == R and gsm == sm
    finally:
        cs.cs_set_free(s)


# ----------------------------------------------------------- error handling
def test_errors(cs, ctx):
    with pytest.raises(cs.CsError):
        cs.cs_sprinkle(ctx, 3, 10, 1)
    with pytest.raises(cs.CsError):
        cs.cs_sprinkle(ctx, 2, -1, 1)
    s = cs.cs_sprinkle(ctx, 2, 100, 1)
    with pytest.raises(cs.CsError):
        cs.cs_interval_abundances(ctx, s, 3, 0)     # not linked
    cs.cs_link(ctx, s)
    with pytest.raises(cs.CsError):
        cs.cs_interval_abundances(ctx, s, 2, 0)     # kmax < 3
    cs.cs_set_free(s)
    small = cs.cs_create(0, 1 << 20, None)          # 1 MiB budget
    try:
        s = cs.cs_sprinkle(small, 2, 4096, 1)        # coords fit, matrix (2 MiB) does not
        with pytest.raises(cs.CsError) as e:
            cs.cs_link(small, s)
        assert e.value.status == 2
        cs.cs_set_free(s)
    finally:
        cs.cs_destroy(small)


def test_deterministic_repeat(cs, ctx):
    out = []
    for _ in range(3):
        s = gpu_set(cs, ctx, 4, 1800, 77)
        out.append(cs.cs_interval_abundances(ctx, s, 3, 0))
        cs.cs_set_free(s)
    assert all(np.array_equal(o[0], out[0][0]) and o[1:] == out[0][1:] for o in out)


# ------------------------------------------------------- full-size workloads
def golden(name):
    with open(GOLDEN) as f:
        g = json.load(f)
    if name not in g:
        pytest.skip("no stored oracle result for %s" % name)
    return g[name]


@pytest.mark.parametrize("path", [0, 1, 2, 3])
@pytest.mark.parametrize("name", ["2d_1024", "4d_16384"])
def test_workload_matches_stored_oracle(cs, ctx, name, path):
    g = golden(name)
    say("case workload %s path=%d" % (name, path))
    s = gpu_set(cs, ctx, g["d"], g["N"], g["seed"])
    try:
        n, R, sm = cs.cs_interval_abundances(ctx, s, 3, path)
        assert [int(x) for x in n] == g["n"] and R == g["R"] and sm == g["summ"]
        S = cs.cs_bd_action(ctx, s)
        assert S == float.fromhex(g["S"])
        import hashlib
        assert hashlib.sha256(cs.cs_get_bitset(ctx, s).tobytes()).hexdigest() == g["bitset_sha256"]
    finally:
        cs.cs_set_free(s)


def test_full_size_2d_131072_against_stored_oracle(cs, ctx):
    """The 2 GiB workload in the launch configuration bench.py times: matrix
    bytes (sha256), abundances, R, sum of m and action equal the stored oracle
    results (tests/golden/make_golden.py --large); the per-row-block
    breakdown sums to the totals, and two sampled row blocks equal the
    oracle's count over the same rows."""
    import hashlib
    g = golden("2d_131072")
    N = g["N"]
    say("case full-size 2D N=%d" % N)
    s = gpu_set(cs, ctx, g["d"], N, g["seed"])
    try:
        bits = cs.cs_get_bitset(ctx, s)
        assert hashlib.sha256(bits.tobytes()).hexdigest() == g["bitset_sha256"]
        for path in (0, 3, 2, 1):
            say("  path %d" % path)
            n, R, sm = cs.cs_interval_abundances(ctx, s, 3, path)
            assert [int(x) for x in n] == g["n"] and R == g["R"] and sm == g["summ"]
        assert cs.cs_bd_action(ctx, s) == float.fromhex(g["S"])
        blocks = cs.cs_interval_abundances_rows(ctx, s, 3, 0)
        tot = blocks.sum(axis=0)
        assert [int(x) for x in tot[:4]] == g["n"] and int(tot[4]) == g["R"] and int(tot[5]) == g["summ"]
        for b in (0, blocks.shape[0] // 2 + 7):
            say("  oracle row block %d" % b)
            h, R, sm = oracle.count_bits(bits, N, nbins=4, rows=(b * 256, b * 256 + 256))
            assert list(blocks[b, :4]) == list(h) and blocks[b, 4] == R and blocks[b, 5] == sm
    finally:
        cs.cs_set_free(s)


@pytest.mark.parametrize("path", [1, 2, 3])
@pytest.mark.parametrize("d,N,seed", [(2, 9000, 61), (4, 9500, 62)])
def test_full_histogram_beyond_lds_bins(cs, ctx, d, N, seed, path):
    """kmax = N-2 > 8191: small sizes are binned in LDS, larger ones with
    device atomics; the whole histogram equals the oracle's."""
    say("case fullhist N-2 d=%d N=%d path=%d" % (d, N, path))
    s = gpu_set(cs, ctx, d, N, seed)
    try:
        n, R, sm = cs.cs_interval_abundances(ctx, s, N - 2, path)
        oc, _, _ = oracle.sprinkle(d, N, seed)
        h, oR, osm = oracle.count_bits(oracle.link(d, oc), N, nbins=N - 1)
        assert np.array_equal(n, h) and R == oR and sm == osm
    finally:
        cs.cs_set_free(s)


@pytest.mark.parametrize("eps", [1.0, 0.5, 2.0**-6])
@pytest.mark.parametrize("N,seed", [(300, 71), (2048, 72), (5000, 73)])
def test_smeared_action_matches_oracle(cs, ctx, N, seed, eps):
    say("case smeared N=%d eps=%r" % (N, eps))
    s = gpu_set(cs, ctx, 2, N, seed)
    try:
        S = cs.cs_smeared_action(ctx, s, eps)
        oc, _, _ = oracle.sprinkle(2, N, seed)
        h, _, _ = oracle.count_bits(oracle.link(2, oc), N, nbins=N - 1)
        So = oracle.smeared_action(N, h, eps)
        assert S == So, (S, So)
        if eps == 1.0:
            assert S == cs.cs_bd_action(ctx, s)
    finally:
        cs.cs_set_free(s)


def test_smeared_action_rejects_bad_arguments(cs, ctx):
    s = gpu_set(cs, ctx, 4, 100, 1)
    with pytest.raises(cs.CsError):
        cs.cs_smeared_action(ctx, s, 0.5)          # 4D
    cs.cs_set_free(s)
    s = gpu_set(cs, ctx, 2, 100, 1)
    for bad in (0.0, -0.1, 1.5):
        with pytest.raises(cs.CsError):
            cs.cs_smeared_action(ctx, s, bad)
    cs.cs_set_free(s)
