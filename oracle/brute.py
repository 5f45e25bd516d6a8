"""Pure-Python brute force for tiny causal sets.

TEST INFRASTRUCTURE.  Used only to pin the C oracle on small inputs: every
quantity is recomputed here from its definition with Python loops and Python
floats (IEEE binary64, one rounding per operation, no fused multiply-add).

* relation: timelike separation in flat 2D light-cone or 4D Cartesian
  coordinates (Sec. 1.1 of arXiv:1709.03013);
* interval abundances: for each related pair the number of elements related
  to both, counted over all k (no index-range shortcut, so a wrong topological
  order or a wrong mask in the C oracle would show);
* 2D orders from permutations (the random 2D orders of Sec. 1 of the paper).
"""
from __future__ import annotations

import itertools
from typing import Sequence


def related(d: int, coords: Sequence[Sequence[float]], i: int, j: int) -> bool:
    """i precedes j (strictly timelike, i earlier)."""
    if d == 2:
        u, v = coords[0], coords[1]
        return u[i] < u[j] and v[i] < v[j]
    t, x, y, z = coords
    dt = t[j] - t[i]
    dx = x[j] - x[i]
    dy = y[j] - y[i]
    dz = z[j] - z[i]
    return dt > 0.0 and dt * dt > (dx * dx + dy * dy) + dz * dz


def precedes_matrix(d: int, coords) -> list[list[bool]]:
    """P[a][b] = a precedes b, for every ordered pair, by the coordinates alone."""
    N = len(coords[0])
    P = [[False] * N for _ in range(N)]
    for a in range(N):
        for b in range(N):
            if a != b:
                # the relation is defined with the earlier element first
                P[a][b] = related(d, coords, a, b)
    return P


def abundances_from_precedes(P: list[list[bool]]):
    """Full histogram of interval sizes over related pairs, R and sum of m.

    m(a,b) = #{c : a<c and c<b in the order} for every a<b in the order.
    """
    N = len(P)
    hist = [0] * max(N - 1, 1)
    R = 0
    summ = 0
    for a in range(N):
        for b in range(N):
            if not P[a][b]:
                continue
            m = sum(1 for c in range(N) if P[a][c] and P[c][b])
            hist[m] += 1
            R += 1
            summ += m
    return hist, R, summ


def abundances(d: int, coords):
    return abundances_from_precedes(precedes_matrix(d, coords))


def order2d_from_perm(perm: Sequence[int]) -> list[list[bool]]:
    """The 2D order of a permutation: a precedes b iff a<b and perm[a]<perm[b]."""
    N = len(perm)
    return [[(a < b and perm[a] < perm[b]) for b in range(N)] for a in range(N)]


def all_2d_orders(N: int):
    for perm in itertools.permutations(range(N)):
        yield perm, order2d_from_perm(perm)


def bd_action_2d(N: int, n: Sequence[int]) -> float:
    """Eq. 4 with n_i (i = 1, 2, 3) = pairs with i-1 interior elements."""
    return 2.0 * float(N - 2 * n[0] + 4 * n[1] - 2 * n[2])


def pack_rows(P_sym: list[list[bool]]) -> list[list[int]]:
    """Pack a symmetric boolean matrix into 64-bit words, LSB first, rows padded
    to a multiple of 4 words."""
    N = len(P_sym)
    W = ((N + 63) // 64 + 3) // 4 * 4
    rows = []
    for i in range(N):
        words = [0] * W
        for k in range(N):
            if P_sym[i][k]:
                words[k // 64] |= 1 << (k % 64)
        rows.append(words)
    return rows
