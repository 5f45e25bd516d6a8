"""Pins for the oracle's (1+1) de Sitter slab (Sec. 6.1, Eq. 9) on the CPU.

* the sprinkle against an independent numpy construction (numpy's Philox,
  rejection in the unit disk, sort by w = tan(eta));
* the relation, written with tangents of differences, against the paper's
  own condition pi - |pi - |theta_1 - theta_2|| < |eta_1 - eta_2| evaluated
  with arctan / arctan2 (only pairs within rounding of the light cone may
  differ);
* transitivity and orientation of the relation (a partial order compatible
  with the label order);
* the ordering fraction against its closed form as an integral over the
  density sec^2(eta) / (2 tan eta0): for a uniform angle difference the
  geodesic distance is uniform on [0, pi], so P(related) = E|eta_1 - eta_2| / pi;
* the mean number of Philox blocks per element against 4/pi (acceptance in
  the unit disk).
"""
import math

import numpy as np
import pytest
from scipy import integrate

U64 = 2**64
ETA0 = 0.5


def numpy_block(seed, c, a):
    cval = c + (a << 64)
    g = np.random.Philox(key=[seed % U64, 5], counter=(cval - 1) % 2**256)
    return g.random_raw(4)


def numpy_sprinkle(N, seed, w0):
    w = np.zeros(N)
    x = np.zeros(N)
    y = np.zeros(N)
    drawn = 0
    for c in range(N):
        for a in range(64):
            r = numpy_block(seed, c, a)
            drawn += 1
            d = (r >> np.uint64(11)).astype(np.float64) * 2.0**-53
            wc = (2.0 * d[0] - 1.0) * w0
            xc = 2.0 * d[1] - 1.0
            yc = 2.0 * d[2] - 1.0
            rr = xc * xc + yc * yc
            w[c] = wc
            if 0.0 < rr < 1.0:
                x[c], y[c] = xc, yc
                break
    order = np.lexsort((np.arange(N), w))
    return w[order], x[order], y[order], order, drawn


@pytest.mark.parametrize("N,seed", [(0, 1), (1, 3), (2, 4), (300, 7), (1500, 11)])
def test_sprinkle_matches_numpy(oracle_lib, N, seed):
    coords, orig, drawn = oracle_lib.sprinkle_desitter(N, seed, ETA0)
    w, x, y, order, ref_drawn = numpy_sprinkle(N, seed, math.tan(ETA0))
    assert drawn == ref_drawn
    assert np.array_equal(orig, order)
    assert np.array_equal(coords[0], w)
    assert np.array_equal(coords[1], x)
    assert np.array_equal(coords[2], y)


def test_sprinkle_support_and_order(oracle_lib):
    N = 50000
    coords, _, drawn = oracle_lib.sprinkle_desitter(N, 21, ETA0)
    w0 = math.tan(ETA0)
    w, x, y = coords
    assert np.all(np.diff(w) >= 0)
    assert np.all(np.abs(w) <= w0)
    r2 = x * x + y * y
    assert np.all((r2 > 0) & (r2 < 1))
    # w uniform on [-w0, w0]; angle uniform on [0, 2 pi)
    se = w0 / math.sqrt(3 * N)
    assert abs(w.mean()) < 6 * se
    th = np.arctan2(y, x)
    assert abs(np.cos(th).mean()) < 6 / math.sqrt(2 * N)
    assert abs(np.sin(th).mean()) < 6 / math.sqrt(2 * N)
    # acceptance of the unit disk in its square is pi / 4
    p = math.pi / 4
    mean, sd = 1 / p, math.sqrt((1 - p) / p**2 / N)
    assert abs(drawn / N - mean) < 6 * sd


def paper_relation(coords):
    """Sec. 6.1: related iff pi - |pi - |theta_1 - theta_2|| < |eta_1 - eta_2|.
    Returns (relation, margin) for all pairs i < j (upper triangle flattened)."""
    eta = np.arctan(coords[0])
    th = np.mod(np.arctan2(coords[2], coords[1]), 2 * np.pi)
    N = coords.shape[1]
    iu, ju = np.triu_indices(N, 1)
    dth = np.abs(th[iu] - th[ju])
    geo = np.pi - np.abs(np.pi - dth)
    margin = np.abs(eta[iu] - eta[ju]) - geo
    return margin > 0, margin, iu, ju


def bits_upper(bits, iu, ju):
    return ((bits[iu, ju >> 6] >> (ju & 63).astype(np.uint64)) & np.uint64(1)).astype(bool)


@pytest.mark.parametrize("seed", [2, 3])
def test_relation_matches_paper_condition(oracle_lib, seed):
    coords, _, _ = oracle_lib.sprinkle_desitter(2000, seed, ETA0)
    bits = oracle_lib.link_desitter(coords)
    rel, margin, iu, ju = paper_relation(coords)
    mine = bits_upper(bits, iu, ju)
    differ = mine != rel
    assert np.all(np.abs(margin[differ]) < 1e-12)
    assert differ.sum() <= 2
    # symmetric packed matrix, zero diagonal
    lo = bits_upper(bits, ju, iu)
    assert np.array_equal(lo, mine)
    N = coords.shape[1]
    assert not any((bits[i, i >> 6] >> np.uint64(i & 63)) & np.uint64(1) for i in range(N))


def test_related_single_pairs(oracle_lib):
    # two elements at the same angle are related iff their times differ
    c = np.array([[-0.3, 0.2, 0.2], [0.5, 0.25, -0.5], [0.0, 0.0, 0.0]])
    assert oracle_lib.related_desitter(c, 0, 1)      # same direction, dw != 0
    assert not oracle_lib.related_desitter(c, 1, 2)  # equal w
    assert not oracle_lib.related_desitter(c, 0, 2)  # opposite directions: dot < 0
    # angle pi/2 apart needs |deta| > pi/2, impossible below eta0 = pi/4
    c = np.array([[-0.9, 0.9], [1.0, 0.0], [0.0, 1.0]])
    assert not oracle_lib.related_desitter(c, 0, 1)
    # small angle, large time gap: related; and its mirror in x
    c = np.array([[-0.5, 0.5], [1.0, 1.0], [0.0, 0.1]])
    assert oracle_lib.related_desitter(c, 0, 1)
    c2 = c.copy()
    c2[2] = -c2[2]
    assert oracle_lib.related_desitter(c2, 0, 1)


def test_relation_is_a_partial_order(oracle_lib):
    coords, _, _ = oracle_lib.sprinkle_desitter(700, 9, ETA0)
    bits = oracle_lib.link_desitter(coords)
    N = coords.shape[1]
    A = np.zeros((N, N), dtype=np.int64)
    for i in range(N):
        row = np.unpackbits(bits[i].view(np.uint8), bitorder="little")[:N]
        A[i] = row
    U = np.triu(A, 1)
    assert np.array_equal(U + U.T, A)
    two = (U @ U) > 0
    assert not np.any(two & (U == 0))          # i < k < j, i~k, k~j  =>  i~j


def ordering_fraction_exact(eta0):
    w0 = math.tan(eta0)

    def f(w2, w1):
        return abs(math.atan(w1) - math.atan(w2)) / math.pi

    lo = integrate.dblquad(f, -w0, w0, lambda w1: -w0, lambda w1: w1, epsabs=1e-12)[0]
    return 2 * lo / (2 * w0) ** 2


def test_ordering_fraction_closed_form(oracle_lib):
    exact = ordering_fraction_exact(ETA0)
    N = 6000
    fr = []
    for seed in range(4):
        coords, _, _ = oracle_lib.sprinkle_desitter(N, 100 + seed, ETA0)
        bits = oracle_lib.link_desitter(coords)
        R = int(np.unpackbits(bits.view(np.uint8)).sum()) // 2
        fr.append(R / (N * (N - 1) / 2))
    # one set's fraction scatters by about 1e-3 at this size (a U-statistic,
    # O(1/sqrt(N))); 3e-3 is several standard deviations of the mean of four
    assert abs(np.mean(fr) - exact) < 3e-3
    assert 0.05 < exact < 0.2


def test_small_eta0_limit_is_flat(oracle_lib):
    """eta0 -> 0: tan eta ~ eta, so the relation becomes the flat cylinder's
    |dt| > angle; with the angle spread over 2 pi and |dt| tiny the set is
    almost an antichain: fraction E|dt| / pi with dt of two U(-eta0, eta0)."""
    eta0 = 0.01
    N = 4000
    coords, _, _ = oracle_lib.sprinkle_desitter(N, 5, eta0)
    bits = oracle_lib.link_desitter(coords)
    R = int(np.unpackbits(bits.view(np.uint8)).sum()) // 2
    frac = R / (N * (N - 1) / 2)
    flat = (2 * eta0 / 3) / math.pi        # E|U1 - U2| = (2 eta0) / 3
    assert abs(frac - flat) < 0.15 * flat
    assert abs(ordering_fraction_exact(eta0) - flat) < 1e-3 * flat
