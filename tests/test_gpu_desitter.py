"""GPU parity for the (1+1) de Sitter slab (Sec. 6.1): sprinkle, sort, link,
counts, BD and smeared actions, called through the C ABI, against the oracle.

Coordinates and matrix words bit-exact; abundances, R and the sum of
interior counts bit-exact; both actions bit-identical (one rounding of an
exact integer bracket, or the same fixed-order sum on both sides)."""
import math
import sys

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

ETA0 = 0.5
EPS = 2.0**-6


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


@pytest.mark.parametrize("N,seed,eta0", [(0, 1, ETA0), (1, 2, ETA0), (2, 3, ETA0), (65, 4, ETA0),
                                         (2047, 5, ETA0), (2049, 6, ETA0), (6000, 7, ETA0),
                                         (3000, 8, 0.05), (3000, 9, 0.78)])
def test_sprinkle_and_link_match_oracle(cs, ctx, N, seed, eta0):
    say("case desitter sprinkle+link N=%d seed=%d eta0=%g" % (N, seed, eta0))
    s = cs.cs_sprinkle_desitter(ctx, N, seed, eta0)
    try:
        assert cs.cs_set_manifold(s) == (cs.CS_MANIFOLD_DESITTER, 3)
        assert cs.cs_set_info(s)[0] == 2
        coords, orig = cs.cs_get_coords(ctx, s)
        oc, oo, _ = oracle.sprinkle_desitter(N, seed, eta0)
        assert np.array_equal(coords.view(np.uint64), oc.view(np.uint64))
        assert np.array_equal(orig, oo)
        cs.cs_link(ctx, s)
        bits = cs.cs_get_bitset(ctx, s)
        assert np.array_equal(bits, oracle.link_desitter(oc))
    finally:
        cs.cs_set_free(s)


@pytest.mark.parametrize("path", [1, 2, 3])
@pytest.mark.parametrize("N,seed", [(300, 11), (2500, 12), (7000, 13)])
def test_counts_and_actions_match_oracle(cs, ctx, N, seed, path):
    say("case desitter counts N=%d path=%d" % (N, path))
    s = cs.cs_sprinkle_desitter(ctx, N, seed, ETA0)
    try:
        cs.cs_link(ctx, s)
        n, R, sm = cs.cs_interval_abundances(ctx, s, N - 2, path)
        oc, _, _ = oracle.sprinkle_desitter(N, seed, ETA0)
        h, oR, osm = oracle.count_bits(oracle.link_desitter(oc), N, nbins=N - 1)
        assert np.array_equal(n, h) and R == oR and sm == osm
        assert cs.cs_bd_action(ctx, s) == oracle.bd_action(2, N, h[:4])
        assert cs.cs_smeared_action(ctx, s, EPS) == oracle.smeared_action(N, h, EPS)
    finally:
        cs.cs_set_free(s)


def test_full_size_sampled_row_blocks(cs, ctx):
    """N = 2^15 at eta0 = 0.5, the size of the paper's abundance figure:
    the whole matrix against the oracle's, and sampled 256-row blocks of
    the full histogram against the oracle's count over those rows."""
    N, seed = 32768, 21
    say("case desitter full size N=%d" % N)
    s = cs.cs_sprinkle_desitter(ctx, N, seed, ETA0)
    try:
        cs.cs_link(ctx, s)
        oc, _, _ = oracle.sprinkle_desitter(N, seed, ETA0)
        obits = oracle.link_desitter(oc)
        assert np.array_equal(cs.cs_get_bitset(ctx, s), obits)
        kmax = 300
        blocks = cs.cs_interval_abundances_rows(ctx, s, kmax, 0)
        for b in (0, 17, 64, 101, 127):
            lo, hi = b * 256, min(b * 256 + 256, N)
            h, R, sm = oracle.count_bits(obits, N, nbins=kmax + 1, rows=(lo, hi))
            assert list(blocks[b, :kmax + 1]) == list(h) and blocks[b, kmax + 1] == R
            assert blocks[b, kmax + 2] == sm
    finally:
        cs.cs_set_free(s)


@pytest.mark.parametrize("N,seed", [(3000, 41), (513, 42), (1024, 43)])
def test_link_ragged_sizes_match_oracle(cs, ctx, N, seed):
    say("case desitter link N=%d" % N)
    s = cs.cs_sprinkle_desitter(ctx, N, seed, ETA0)
    try:
        cs.cs_link(ctx, s)
        oc, _, _ = oracle.sprinkle_desitter(N, seed, ETA0)
        assert np.array_equal(cs.cs_get_bitset(ctx, s), oracle.link_desitter(oc))
    finally:
        cs.cs_set_free(s)


def test_rejects_bad_eta0(cs, ctx):
    for bad in (0.0, -0.1, math.pi / 4, 1.0, float("nan")):
        with pytest.raises(cs.CsError):
            cs.cs_sprinkle_desitter(ctx, 100, 1, bad)
