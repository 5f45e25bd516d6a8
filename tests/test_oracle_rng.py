"""Pins for the oracle's random numbers and sprinkling (CPU only).

* Philox4x64-10 against numpy's Philox bit generator (a library routine);
* the sprinkled coordinates against an independent numpy construction;
* statistics fixed by the mathematics: uniform means, the 4D acceptance
  probability pi/24 (volume of the height-1 diamond inside its bounding box),
  topological order of the sorted labels.
"""
import math

import numpy as np
import pytest

U64 = 2**64


def numpy_blocks(key0, tag, n):
    """Philox blocks for counters 0..n-1 (numpy advances before each block)."""
    g = np.random.Philox(key=[key0 % U64, tag], counter=2**256 - 1)
    return g.random_raw(4 * n).reshape(n, 4)


@pytest.mark.parametrize("ctr", [0, 1, 2, 63, 64, 2**32 - 1, 2**32, 2**63 + 5, 2**64 - 1])
@pytest.mark.parametrize("key", [(0, 0), (1, 1), (3, 2), (2**64 - 1, 2**64 - 1), (0x0123456789ABCDEF, 7)])
def test_philox_matches_numpy(oracle_lib, ctr, key):
    mine = oracle_lib.philox4x64_10([ctr, 0, 0, 0], key)
    g = np.random.Philox(key=list(key), counter=(ctr - 1) % 2**256)
    ref = g.random_raw(4)
    assert [int(x) for x in mine] == [int(x) for x in ref]


def test_philox_full_counter_words(oracle_lib):
    # All four counter words enter the rounds.
    c = [5, 2**40 + 3, 17, 2**63]
    mine = oracle_lib.philox4x64_10(c, (9, 2))
    cval = c[0] + (c[1] << 64) + (c[2] << 128) + (c[3] << 192)
    g = np.random.Philox(key=[9, 2], counter=cval - 1)
    assert [int(x) for x in mine] == [int(x) for x in g.random_raw(4)]


@pytest.mark.parametrize("N,seed", [(1, 0), (2, 9), (257, 1), (1024, 1), (5000, 77)])
def test_sprinkle_2d_matches_numpy(oracle_lib, N, seed):
    coords, orig, drawn = oracle_lib.sprinkle(2, N, seed)
    assert drawn == N
    r = numpy_blocks(seed, 1, N)
    a = r[:, 0] >> np.uint64(11)
    b = r[:, 1] >> np.uint64(11)
    order = np.lexsort((np.arange(N), a, a + b))
    u = a.astype(np.float64) * 2.0**-53
    v = b.astype(np.float64) * 2.0**-53
    assert np.array_equal(orig, order)
    assert np.array_equal(coords[0], u[order])
    assert np.array_equal(coords[1], v[order])


@pytest.mark.parametrize("N,seed", [(1, 3), (100, 2), (3000, 12)])
def test_sprinkle_4d_matches_numpy(oracle_lib, N, seed):
    coords, orig, drawn = oracle_lib.sprinkle(4, N, seed)
    r = numpy_blocks(seed, 2, drawn)
    t = (r[:, 0] >> np.uint64(11)).astype(np.float64) * 2.0**-53
    x = (r[:, 1] >> np.uint64(11)).astype(np.float64) * 2.0**-53 - 0.5
    y = (r[:, 2] >> np.uint64(11)).astype(np.float64) * 2.0**-53 - 0.5
    z = (r[:, 3] >> np.uint64(11)).astype(np.float64) * 2.0**-53 - 0.5
    m = np.minimum(t, 1.0 - t)
    acc = ((x * x + y * y) + z * z) < m * m
    assert acc.sum() == N and acc[-1]          # exactly N accepted, the last draw accepted
    idx = np.nonzero(acc)[0]
    kt = r[idx, 0] >> np.uint64(11)
    order = np.lexsort((np.arange(N), kt))
    assert np.array_equal(orig, order)
    for q, arr in enumerate((t, x, y, z)):
        assert np.array_equal(coords[q], arr[idx][order])


def test_sprinkle_uniform_means(oracle_lib):
    coords, _, _ = oracle_lib.sprinkle(2, 200000, 5)
    se = math.sqrt(1 / 12 / 200000)
    assert abs(coords[0].mean() - 0.5) < 6 * se
    assert abs(coords[1].mean() - 0.5) < 6 * se
    c4, _, drawn = oracle_lib.sprinkle(4, 100000, 6)
    # spatial coordinates are symmetric about 0, time about 1/2
    assert abs(c4[1].mean()) < 0.01 and abs(c4[2].mean()) < 0.01 and abs(c4[3].mean()) < 0.01
    assert abs(c4[0].mean() - 0.5) < 0.01


def test_acceptance_probability_is_pi_over_24(oracle_lib):
    N = 200000
    _, _, drawn = oracle_lib.sprinkle(4, N, 123)
    p = math.pi / 24
    se = math.sqrt(p * (1 - p) / drawn)
    assert abs(N / drawn - p) < 6 * se


def test_sprinkle_inside_region(oracle_lib):
    c2, _, _ = oracle_lib.sprinkle(2, 10000, 8)
    assert (c2 >= 0).all() and (c2 < 1).all()
    c4, _, _ = oracle_lib.sprinkle(4, 10000, 8)
    t, x, y, z = c4
    r = np.sqrt(x * x + y * y + z * z)
    assert (r <= np.minimum(t, 1 - t) + 1e-15).all()


@pytest.mark.parametrize("d", [2, 4])
def test_sorted_order_is_topological(oracle_lib, d):
    from oracle import brute
    coords, _, _ = oracle_lib.sprinkle(d, 300, 21)
    lists = [list(map(float, c)) for c in coords]
    N = 300
    for a in range(N):
        for b in range(N):
            if a != b and brute.related(d, lists, a, b):
                assert a < b
    if d == 4:
        assert (np.diff(coords[0]) >= 0).all()
    else:
        s = coords[0] + coords[1]
        assert (np.diff(s) >= -1e-15).all()


def test_seeds_give_distinct_sets(oracle_lib):
    a, _, _ = oracle_lib.sprinkle(2, 64, 1)
    b, _, _ = oracle_lib.sprinkle(2, 64, 2)
    assert not np.array_equal(a, b)
    c, _, _ = oracle_lib.sprinkle(2, 64, 1)
    assert np.array_equal(a, c)
