"""Pins for the oracle's smeared action (Eq. 5), CPU only.

* eps = 1 reduces Eq. 5 to Eq. 4 exactly (f2(0,1) = 1, f2(1,1) = -2,
  f2(2,1) = 1, f2(k>=3,1) = 0);
* for dyadic eps the oracle's double result matches Eq. 5 evaluated in exact
  rational arithmetic, written as the paper prints it (with the divisions by
  1 - eps), not in the oracle's multiplied-out form.
"""
from fractions import Fraction

import numpy as np
import pytest


def f2_exact(k, eps):
    """Eq. 5's f2, exactly, as printed."""
    e = Fraction(eps)
    q = 1 - e
    return q**k * (1 - 2 * e * k / q + e * e * k * (k - 1) / (2 * q * q))


def smeared_exact(N, hist, eps):
    e = Fraction(eps)
    s = sum(int(h) * f2_exact(k, eps) for k, h in enumerate(hist))
    return 2 * e * (N - 2 * e * s)


@pytest.mark.parametrize("seed", range(5))
def test_eps_one_is_eq4(oracle_lib, seed):
    rng = np.random.default_rng(seed)
    N = int(rng.integers(10, 5000))
    hist = rng.integers(0, 10**6, size=int(rng.integers(3, 50))).astype(np.uint64)
    S = oracle_lib.smeared_action(N, hist, 1.0)
    n = [int(x) for x in hist[:3]]
    assert S == 2.0 * (N - 2 * n[0] + 4 * n[1] - 2 * n[2])


@pytest.mark.parametrize("eps", [0.75, 0.5, 0.125, 2.0**-6])
@pytest.mark.parametrize("d,N,seed", [(2, 64, 1), (2, 300, 2), (2, 700, 3)])
def test_matches_exact_rational_eq5(oracle_lib, eps, d, N, seed):
    coords, _, _ = oracle_lib.sprinkle(d, N, seed)
    hist, _, _ = oracle_lib.count_bits(oracle_lib.link(d, coords), N, nbins=N - 1)
    exact = smeared_exact(N, hist, eps)
    got = oracle_lib.smeared_action(N, hist, eps)
    # rounding of O(N) terms of size up to ~N: bound the absolute error by
    # a few ulps of the largest partial sum
    scale = 2 * eps * max(N, float(np.max(hist)) * N)
    assert abs(got - float(exact)) <= 1e-13 * scale


def test_chain_smeared_reduces_at_eps_one(oracle_lib):
    import causet_inputs as ci
    N = 200
    hist, _, _ = oracle_lib.count_bits(ci.pack_symmetric(ci.chain_order(N)), N, nbins=N - 1)
    assert oracle_lib.smeared_action(N, hist, 1.0) == 2.0 * N
