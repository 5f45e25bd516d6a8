"""Pins for the oracle's relation and packed matrix (CPU only).

* the matrix equals a pure-Python brute force of the timelike relation;
* structural invariants: symmetric, zero diagonal, zero padding, LSB-first;
* the 2D ordering fraction: a 2D order is a random permutation, so R is the
  number of non-inversions, E[R] = N(N-1)/4 and Var R = N(N-1)(2N+5)/72;
* the 4D ordering fraction of a flat diamond: E[R]/C(N,2) = 1/10
  (Myrheim-Meyer, d = 4).
"""
import math

import numpy as np
import pytest

import causet_inputs as ci
from oracle import brute


def unpack(bits, N):
    by = bits.view(np.uint8).reshape(N, -1)
    return np.unpackbits(by, axis=1, bitorder="little").astype(bool)


@pytest.mark.parametrize("d,N,seed", [(2, 1, 1), (2, 2, 4), (2, 63, 1), (2, 64, 2), (2, 65, 3),
                                      (2, 130, 4), (4, 1, 5), (4, 70, 6), (4, 129, 7)])
def test_link_matches_brute_force(oracle_lib, d, N, seed):
    coords, _, _ = oracle_lib.sprinkle(d, N, seed)
    bits = oracle_lib.link(d, coords)
    W = ci.row_words(N)
    assert bits.shape == (N, W) and W % 4 == 0
    P = brute.precedes_matrix(d, [list(map(float, c)) for c in coords])
    sym = np.array(P) | np.array(P).T
    full = unpack(bits, N)
    assert np.array_equal(full[:, :N], sym)
    assert not full[:, N:].any()          # padding stays zero
    assert not np.diagonal(full[:, :N]).any()


def test_link_packing_matches_reference_packer(oracle_lib):
    coords = ci.chain_coords(2, 150)
    bits = oracle_lib.link(2, coords)
    assert np.array_equal(bits, ci.pack_symmetric(ci.chain_order(150)))
    coords = ci.antichain_coords(4, 70)
    assert not oracle_lib.link(4, coords).any()
    coords = ci.chain_coords(4, 70)
    assert np.array_equal(oracle_lib.link(4, coords), ci.pack_symmetric(ci.chain_order(70)))


def test_2d_relation_count_distribution(oracle_lib):
    N, S = 64, 400
    Rs = []
    for s in range(S):
        coords, _, _ = oracle_lib.sprinkle(2, N, 1000 + s)
        bits = oracle_lib.link(2, coords)
        Rs.append(int(sum(bin(int(w)).count("1") for w in bits.ravel())) // 2)
    Rs = np.array(Rs, dtype=np.float64)
    mean = N * (N - 1) / 4
    var = N * (N - 1) * (2 * N + 5) / 72
    assert abs(Rs.mean() - mean) < 5 * math.sqrt(var / S)
    # sample variance within a loose chi-square band
    assert 0.7 * var < Rs.var(ddof=1) < 1.4 * var


def test_2d_relation_count_matches_inversions(oracle_lib):
    # R equals the number of non-inversions of v read in u order.
    coords, orig, _ = oracle_lib.sprinkle(2, 500, 31)
    bits = oracle_lib.link(2, coords)
    R = int(np.unpackbits(bits.view(np.uint8), bitorder="little").sum()) // 2
    order = np.argsort(coords[0], kind="stable")
    v = coords[1][order]
    noninv = sum(int((v[a + 1:] > v[a]).sum()) for a in range(500))
    assert R == noninv


def test_4d_ordering_fraction(oracle_lib):
    N, S = 96, 150
    fr = []
    for s in range(S):
        coords, _, _ = oracle_lib.sprinkle(4, N, 5000 + s)
        bits = oracle_lib.link(4, coords)
        R = int(np.unpackbits(bits.view(np.uint8), bitorder="little").sum()) // 2
        fr.append(R / (N * (N - 1) / 2))
    fr = np.array(fr)
    se = fr.std(ddof=1) / math.sqrt(S)
    assert abs(fr.mean() - 0.1) < 5 * se


def test_related_is_strict(oracle_lib):
    # equal coordinates and null separations are unrelated
    c = np.array([[0.25, 0.25, 0.5], [0.25, 0.5, 0.5]])
    assert not oracle_lib.related(2, c, 0, 1)   # equal u
    assert oracle_lib.related(2, c, 0, 2)
    assert not oracle_lib.related(2, c, 1, 2)   # equal v
    c4 = np.array([[0.25, 0.5, 0.5], [0.0, 0.25, 0.0], [0.0, 0.0, 0.0], [0.0, 0.0, 0.0]])
    assert not oracle_lib.related(4, c4, 0, 1)  # null: dt = |dx|
    assert oracle_lib.related(4, c4, 0, 2)
