"""Pins for the oracle's interval abundances and BD action (CPU only).

What fixes the expected values, independently of the oracle's code:
* pure-Python brute force over all triples (tiny sets);
* a library matrix product: with U the strictly upper-triangular 0/1 matrix
  of the order, (U @ U)[i, j] is the number of elements between i and j;
* closed forms: chain (N-1-k intervals of size k), antichain (none), complete
  layered orders, additivity over disjoint unions;
* exact expectations over all 2D orders of N elements (a rational closed
  form, derived below from the product density of two uniform spacings),
  compared with the oracle run on every permutation;
* the 3-chain identity: sum of m over related pairs = sum over k of
  #below(k) * #above(k) for a transitive relation;
* the action of a chain and of an antichain, and of hand-counted layered
  orders; Eq. 4's 2D weights as printed; the 4D weights (the reading of the
  cited BD reference) and their index convention by the moment identities
  that Eq. 4's weights satisfy in 2D, written for d = 4.
"""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

import causet_inputs as ci
from oracle import brute


def unpack(bits, N):
    by = bits.view(np.uint8).reshape(N, -1)
    return np.unpackbits(by, axis=1, bitorder="little")[:, :N].astype(np.float64)


def gemm_histogram(bits, N, nbins):
    A = unpack(bits, N)
    U = np.triu(A, 1)
    M = U @ U                                   # exact: entries < 2^53
    iu = np.nonzero(U)
    m = M[iu].astype(np.int64)
    hist = np.bincount(m, minlength=nbins)[:nbins]
    return hist, len(m), int(m.sum())


# ---------------------------------------------------------------- closed forms
@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 63, 64, 65, 127, 128, 129, 200])
def test_chain(oracle_lib, N):
    bits = ci.pack_symmetric(ci.chain_order(N))
    hist, R, s = oracle_lib.count_bits(bits, N)
    exp = [max(N - 1 - k, 0) for k in range(len(hist))]
    assert list(hist) == exp[:len(hist)] or N <= 1
    assert R == N * (N - 1) // 2
    assert s == sum((N - 1 - k) * k for k in range(max(N - 1, 0)))
    for d in (2, 4):
        h1, R1, s1 = oracle_lib.count_coords(d, ci.chain_coords(d, N))
        assert (R1, s1) == (R, s) and np.array_equal(h1, hist)


@pytest.mark.parametrize("N", [1, 5, 64, 100])
def test_antichain(oracle_lib, N):
    bits = ci.pack_symmetric(ci.antichain_order(N))
    hist, R, s = oracle_lib.count_bits(bits, N)
    assert R == 0 and s == 0 and not hist.any()
    for d in (2, 4):
        h, R, s = oracle_lib.count_coords(d, ci.antichain_coords(d, N))
        assert R == 0 and s == 0


@pytest.mark.parametrize("a,b", [(1, 1), (3, 5), (64, 1), (40, 90)])
def test_two_layers(oracle_lib, a, b):
    bits = ci.pack_symmetric(ci.layered_order([a, b]))
    hist, R, s = oracle_lib.count_bits(bits, a + b)
    assert hist[0] == a * b and hist[1:].sum() == 0 and R == a * b and s == 0


@pytest.mark.parametrize("a,b,c", [(1, 1, 1), (2, 3, 4), (30, 50, 70), (1, 130, 1)])
def test_three_layers(oracle_lib, a, b, c):
    N = a + b + c
    bits = ci.pack_symmetric(ci.layered_order([a, b, c]))
    hist, R, s = oracle_lib.count_bits(bits, N)
    exp = np.zeros(len(hist), dtype=np.int64)
    exp[0] += a * b + b * c
    exp[b] += a * c
    assert np.array_equal(hist, exp)
    assert R == a * b + b * c + a * c and s == a * c * b


def test_disjoint_union_is_additive(oracle_lib):
    o1 = ci.random_dag_order(70, 0.08, 1)
    o2 = ci.layered_order([5, 9, 3])
    o3 = ci.chain_order(40)
    N = 70 + 17 + 40
    u = ci.disjoint_union(o1, o2, o3)
    h, R, s = oracle_lib.count_bits(ci.pack_symmetric(u), N, nbins=N)
    tot = np.zeros(N, dtype=np.int64)
    Rt = st = 0
    for o in (o1, o2, o3):
        n = o.shape[0]
        hh, RR, ss = oracle_lib.count_bits(ci.pack_symmetric(o), n, nbins=N)
        tot += hh.astype(np.int64)
        Rt += RR
        st += ss
    assert np.array_equal(h, tot) and R == Rt and s == st


# -------------------------------------------------------------- brute / gemm
@pytest.mark.parametrize("d,N,seed", [(2, 20, 1), (2, 40, 2), (4, 30, 3), (4, 45, 4)])
def test_tiers_match_brute_force(oracle_lib, d, N, seed):
    coords, _, _ = oracle_lib.sprinkle(d, N, seed)
    hb, Rb, sb = brute.abundances(d, [list(map(float, c)) for c in coords])
    h1, R1, s1 = oracle_lib.count_coords(d, coords)
    bits = oracle_lib.link(d, coords)
    h2, R2, s2 = oracle_lib.count_bits(bits, N)
    assert list(h1) == hb and list(h2) == hb
    assert R1 == R2 == Rb and s1 == s2 == sb


@pytest.mark.parametrize("kind,N,seed", [("2d", 700, 11), ("4d", 900, 12), ("dag", 333, 13),
                                          ("2d", 1024, 1), ("4d", 2048, 14)])
def test_tier2_matches_matrix_product(oracle_lib, kind, N, seed):
    if kind == "dag":
        bits = ci.pack_symmetric(ci.random_dag_order(N, 0.02, seed))
    else:
        d = 2 if kind == "2d" else 4
        coords, _, _ = oracle_lib.sprinkle(d, N, seed)
        bits = oracle_lib.link(d, coords)
    hg, Rg, sg = gemm_histogram(bits, N, N - 1)
    h, R, s = oracle_lib.count_bits(bits, N)
    assert np.array_equal(h, hg) and R == Rg and s == sg


def test_tier1_matches_tier2_medium(oracle_lib):
    for d, N, seed in [(2, 400, 41), (4, 500, 42)]:
        coords, _, _ = oracle_lib.sprinkle(d, N, seed)
        h1, R1, s1 = oracle_lib.count_coords(d, coords)
        h2, R2, s2 = oracle_lib.count_bits(oracle_lib.link(d, coords), N)
        assert np.array_equal(h1, h2) and R1 == R2 and s1 == s2


def test_interval_size_matches_matrix_product(oracle_lib):
    coords, _, _ = oracle_lib.sprinkle(2, 300, 8)
    bits = oracle_lib.link(2, coords)
    U = np.triu(unpack(bits, 300), 1)
    M = U @ U
    rng = np.random.default_rng(0)
    for _ in range(500):
        i, j = sorted(rng.choice(300, 2, replace=False))
        assert oracle_lib.interval_size(bits, i, j) == int(M[i, j])


def test_row_ranges_partition(oracle_lib):
    coords, _, _ = oracle_lib.sprinkle(4, 3000, 5)
    bits = oracle_lib.link(4, coords)
    h, R, s = oracle_lib.count_bits(bits, 3000, nbins=8)
    acc = np.zeros(8, dtype=np.uint64)
    Ra = sa = 0
    for lo in range(0, 3000, 256):
        hh, RR, ss = oracle_lib.count_bits(bits, 3000, nbins=8, rows=(lo, min(lo + 256, 3000)))
        acc += hh
        Ra += RR
        sa += ss
    assert np.array_equal(acc, h) and Ra == R and sa == s


@pytest.mark.parametrize("N,seed", [(1024, 1), (3000, 9)])
def test_three_chain_identity_2d(oracle_lib, N, seed):
    coords, _, _ = oracle_lib.sprinkle(2, N, seed)
    bits = oracle_lib.link(2, coords)
    _, _, s = oracle_lib.count_bits(bits, N)
    assert s == oracle_lib.three_chains(bits, N)


# --------------------------------------------------- exact 2D expectations
def _H(n):
    return sum((Fraction(1, k) for k in range(1, n + 1)), Fraction(0))


def _B(a, b):
    """Beta(a, b) for positive integers."""
    return Fraction(math.factorial(a - 1) * math.factorial(b - 1), math.factorial(a + b - 1))


def expected_abundance_2d(N, k):
    """E[N_k] over random 2D orders of N elements.

    Two uniform points of the unit square are related with probability 1/2;
    given that, the area s of their interval has density
    f(s) = 4[-(1+s) ln s - 2(1-s)] (product of two spacings with density
    2(1-x)), and each other point falls inside with probability s.  Hence
    E[N_k] = C(N,2)/2 C(N-2,k) int f(s) s^k (1-s)^(N-2-k) ds, and with
    int s^a (1-s)^b (-ln s) ds = B(a+1,b+1)(H_{a+b+1} - H_a) this is rational.
    """
    n = N - 2 - k
    if n < 0:
        return Fraction(0)
    I = 4 * (_B(k + 1, n + 1) * (_H(k + n + 1) - _H(k))
             + _B(k + 2, n + 1) * (_H(k + n + 2) - _H(k + 1))
             - 2 * _B(k + 1, n + 2))
    return Fraction(N * (N - 1), 4) * math.comb(N - 2, k) * I


def test_expectation_closed_form_small_values():
    assert [expected_abundance_2d(4, k) for k in range(4)] == [
        Fraction(29, 12), Fraction(1, 2), Fraction(1, 12), Fraction(0)]
    # the total over k is the expected number of related pairs, C(N,2)/2
    for N in (4, 9, 30):
        assert sum(expected_abundance_2d(N, k) for k in range(N - 1)) == Fraction(N * (N - 1), 4)


@pytest.mark.parametrize("N", [3, 4, 5, 6, 7])
def test_oracle_over_all_2d_orders_matches_expectation(oracle_lib, N):
    tot = np.zeros(max(N - 1, 1), dtype=object)
    tot[:] = 0
    S = Fraction(0)
    count = 0
    for perm in itertools.permutations(range(N)):
        coords = ci.perm_coords_2d(perm)
        h, R, s = oracle_lib.count_bits(oracle_lib.link(2, coords), N)
        tot += np.array([int(x) for x in h], dtype=object)
        S += Fraction(oracle_lib.bd_action(2, N, h[:4]))
        count += 1
    for k in range(N - 1):
        assert Fraction(int(tot[k]), count) == expected_abundance_2d(N, k)
    if N >= 4:
        # mean 2D action of a flat diamond: exactly 2 at every N >= 4
        assert S / count == 2
        ES = 2 * (N - 2 * expected_abundance_2d(N, 0) + 4 * expected_abundance_2d(N, 1)
                  - 2 * expected_abundance_2d(N, 2))
        assert ES == 2


def test_large_n_means_match_expectation(oracle_lib):
    N, S = 256, 60
    acc = np.zeros(4)
    for s in range(S):
        coords, _, _ = oracle_lib.sprinkle(2, N, 9000 + s)
        h, _, _ = oracle_lib.count_bits(oracle_lib.link(2, coords), N, nbins=4)
        acc += h.astype(np.float64)
    mean = acc / S
    exp = np.array([float(expected_abundance_2d(N, k)) for k in range(4)])
    assert np.all(np.abs(mean - exp) / exp < 0.05)


# ---------------------------------------------------------------- action
@pytest.mark.parametrize("N", [4, 5, 64, 1000, 131072])
def test_action_chain_and_antichain(oracle_lib, N):
    chain = [N - 1, N - 2, N - 3, N - 4]
    assert oracle_lib.bd_action(2, N, chain) == 2.0 * N
    assert oracle_lib.bd_action(4, N, chain) == (4.0 / math.sqrt(6.0)) * (N - 1)
    assert oracle_lib.bd_action(2, N, [0, 0, 0, 0]) == 2.0 * N
    assert oracle_lib.bd_action(4, N, [0, 0, 0, 0]) == (4.0 / math.sqrt(6.0)) * N


def test_action_matches_brute_eq4(oracle_lib):
    coords, _, _ = oracle_lib.sprinkle(2, 30, 77)
    hb, _, _ = brute.abundances(2, [list(map(float, c)) for c in coords])
    assert oracle_lib.bd_action(2, 30, hb[:4]) == brute.bd_action_2d(30, hb[:4])


def test_action_chain_from_counts(oracle_lib):
    N = 300
    bits = ci.pack_symmetric(ci.chain_order(N))
    h, _, _ = oracle_lib.count_bits(bits, N, nbins=4)
    assert oracle_lib.bd_action(2, N, h) == 2.0 * N


# ------------------------------------------- the action's weights and indices
def _bracket_weights(oracle_lib, d):
    """The integer weights c_k the oracle's action gives N_k (k = 0..3), read
    back from S for N = 0 and a unit abundance vector, and its prefactor
    (S of one isolated element).  S = prefactor * (N + sum_k c_k N_k)."""
    pref = oracle_lib.bd_action(d, 1, [0, 0, 0, 0])
    c = []
    for k in range(4):
        e = [0, 0, 0, 0]
        e[k] = 1
        ratio = oracle_lib.bd_action(d, 0, e) / pref
        assert abs(ratio - round(ratio)) < 1e-12
        c.append(int(round(ratio)))
    return pref, c


def _tau2_moment(c, d, shift=0):
    """sum_k c_k Gamma(k+s+1+2/d) / (Gamma(1+2/d) (k+s)!), exactly, for the
    weights applied to N_{k+s}.  With a Poisson sprinkling of density rho, the
    expected number of intervals of k interior elements in a pair whose
    interval has volume v is weighted by e^{-x} x^k / k! (x = rho v); this sum
    is the integral over x in (0, inf) of x^{2/d} e^{-x} sum_k c_k x^k / k!,
    the moment carrying the squared proper time (v grows as tau^d)."""
    a = Fraction(2, d)
    tot = Fraction(0)
    for k, ck in enumerate(c):
        j = k + shift
        g = Fraction(1)
        for t in range(1, j + 1):           # Gamma(j+1+a) / (Gamma(1+a) j!)
            g *= (t + a) / t
        tot += ck * g
    return tot


def test_action_weights_2d_are_eq4(oracle_lib):
    # Eq. 4 as printed: S = 2 (N - 2 n_1 + 4 n_2 - 2 n_3), n_i = N_{i-1}
    pref, c = _bracket_weights(oracle_lib, 2)
    assert pref == 2.0 and c == [-2, 4, -2, 0]
    # the two moment identities Eq. 4's weights satisfy (d = 2: the squared
    # proper-time moment is sum_k c_k (k+1))
    assert sum(c) == 0
    assert _tau2_moment(c, 2) == 0
    assert sum(ck * (k + 1) for k, ck in enumerate(c)) == 0


def test_action_weights_4d_moments_and_index(oracle_lib):
    """The 4D bracket (reading of the BD weights the paper cites for Eq. 4)
    against identities that fix its index convention: a chain of N elements
    gives N - 1 (sum c_k = 0, sum k c_k = 1), and the d = 4 form of the
    squared-proper-time moment that Eq. 4's weights satisfy in 2D vanishes:
    -1 + 9 (3/2) - 16 (15/8) + 8 (35/16) = 0.  Applied one bin off (to
    N_1..N_4) the same weights give 1/16, so a shifted bracket fails here.  The prefactor 4/sqrt 6 is the
    literature's and stays unpinned by the paper."""
    pref, c = _bracket_weights(oracle_lib, 4)
    assert pref == 4.0 / math.sqrt(6.0)
    assert c == [-1, 9, -16, 8]
    assert sum(c) == 0
    assert sum(k * ck for k, ck in enumerate(c)) == 1
    assert _tau2_moment(c, 4) == 0
    assert _tau2_moment(c, 4, shift=1) == Fraction(1, 16)
    # a sign flip of one weight, or the 2D weights, break it too
    for k in range(4):
        flipped = list(c)
        flipped[k] = -flipped[k]
        assert _tau2_moment(flipped, 4) != 0
    assert _tau2_moment([-2, 4, -2, 0], 4) != 0


def _hand_layered_11211():
    """Complete layered order x1 < x2 < {a, b} < y1 < y2 (layer sizes
    1,1,2,1,1), counted by hand: links x1x2, x2a, x2b, ay1, by1, y1y2 (N_0=6);
    one element inside: x1-a, x1-b (x2), a-y2, b-y2 (y1) (N_1=4); two: x2-y1
    ({a,b}) (N_2=1); three: x1-y1 ({x2,a,b}), x2-y2 ({a,b,y1}) (N_3=2); four:
    x1-y2 (N_4=1).  R = 14 (all 15 pairs but a-b)."""
    return ci.layered_order([1, 1, 2, 1, 1]), [6, 4, 1, 2, 1]


def _hand_boolean_lattice_3():
    """Subsets of {0,1,2} ordered by strict inclusion (8 elements, labels in
    order of size then value): a pair A < B has 2^|B-A| - 2 elements inside.
    |B-A| = 1: 12 pairs (N_0); 2: 6 pairs (N_2); 3: one pair (N_6)."""
    sets = sorted(range(8), key=lambda s: (bin(s).count("1"), s))
    prec = np.array([[a != b and (a & b) == a for b in sets] for a in sets])
    return prec, [12, 0, 6, 0, 0, 0, 1]


@pytest.mark.parametrize("make", [_hand_layered_11211, _hand_boolean_lattice_3])
def test_action_on_hand_counted_orders(oracle_lib, make):
    """Small orders with distinct, hand-counted N_0..N_4: the oracle's counts
    equal the hand counts and its 2D/4D actions equal the brackets written
    out with them, so an index shift (weights on N_1..N_4) changes S here."""
    prec, hand = make()
    N = prec.shape[0]
    h, R, _ = oracle_lib.count_bits(ci.pack_symmetric(prec), N, nbins=len(hand))
    assert [int(x) for x in h] == hand and R == sum(hand)
    n = hand[:4]
    S2 = 2.0 * (N - 2 * n[0] + 4 * n[1] - 2 * n[2])
    K4 = N - n[0] + 9 * n[1] - 16 * n[2] + 8 * n[3]
    assert oracle_lib.bd_action(2, N, h[:4]) == S2
    assert oracle_lib.bd_action(4, N, h[:4]) == (4.0 / math.sqrt(6.0)) * K4
    shifted = N - hand[1] + 9 * hand[2] - 16 * hand[3] + 8 * hand[4]
    assert shifted != K4
