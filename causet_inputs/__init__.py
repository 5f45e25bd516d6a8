"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module holds none of the method's arithmetic: no relation test, no
interval count, no action.  It only builds inputs:

* injected partial orders given combinatorially (chains, antichains, complete
  layered orders, disjoint unions, 2D orders of permutations, random orders
  from the transitive closure of a random DAG), as packed symmetric bitsets
  or as coordinates;
* the ensemble plan (set seeds, sizes, dimensions) for the batched workload;
* the request plan (seeds, sizes, dimensions, Poisson arrival times) for the
  served workload.

Plans draw their randomness from numpy's Philox bit generator; the sprinkled
coordinates themselves are drawn inside each implementation from the seed.
"""
from __future__ import annotations

import math

import numpy as np

U64 = 2**64


def row_words(N: int) -> int:
    """Words per packed row: ceil(N/64) rounded up to a multiple of 4."""
    return ((N + 63) // 64 + 3) // 4 * 4


def pack_symmetric(prec: np.ndarray) -> np.ndarray:
    """Pack a strict order given as a boolean (N, N) matrix, prec[a, b] = a<b
    in the order, into symmetric 64-bit rows (LSB first, zero padding)."""
    prec = np.asarray(prec, dtype=bool)
    N = prec.shape[0]
    sym = prec | prec.T
    np.fill_diagonal(sym, False)
    W = row_words(N)
    padded = np.zeros((N, W * 64), dtype=np.uint8)
    padded[:, :N] = sym
    by = np.packbits(padded.reshape(N, W * 8, 8), axis=2, bitorder="little")
    return by.reshape(N, W * 8).view(np.uint64).reshape(N, W).copy()


def chain_order(N: int) -> np.ndarray:
    return np.triu(np.ones((N, N), dtype=bool), 1)


def antichain_order(N: int) -> np.ndarray:
    return np.zeros((N, N), dtype=bool)


def layered_order(sizes) -> np.ndarray:
    """Complete layered order: every element of layer p precedes every element
    of every later layer q > p."""
    sizes = list(sizes)
    N = sum(sizes)
    lay = np.repeat(np.arange(len(sizes)), sizes)
    return lay[:, None] < lay[None, :]


def disjoint_union(*orders) -> np.ndarray:
    N = sum(o.shape[0] for o in orders)
    out = np.zeros((N, N), dtype=bool)
    s = 0
    for o in orders:
        n = o.shape[0]
        out[s:s + n, s:s + n] = o
        s += n
    return out


def order_2d_from_permutation(perm) -> np.ndarray:
    perm = np.asarray(perm)
    idx = np.arange(perm.size)
    return (idx[:, None] < idx[None, :]) & (perm[:, None] < perm[None, :])


def random_dag_order(N: int, p: float, seed: int) -> np.ndarray:
    """Transitive closure of a random DAG on labels 0..N-1 (edge a->b, a<b,
    with probability p).  Labels are already a linear extension."""
    rng = np.random.Generator(np.random.Philox(key=[seed & (U64 - 1), 11]))
    adj = np.triu(rng.random((N, N)) < p, 1)
    clo = adj.copy()
    for b in range(N - 1, -1, -1):  # successors of b are > b, so their rows are final
        succ = adj[b]
        if succ.any():
            clo[b] |= clo[succ].any(axis=0)
    return clo


def chain_coords(d: int, N: int) -> np.ndarray:
    """A chain placed in the diamond: 2D u_i = v_i = (i+1)/(N+1); 4D on the t axis."""
    s = (np.arange(N, dtype=np.float64) + 1.0) / (N + 1.0)
    if d == 2:
        return np.stack([s, s])
    z = np.zeros(N)
    return np.stack([s, z, z, z])


def antichain_coords(d: int, N: int) -> np.ndarray:
    """An antichain: 2D on the line v = 1 - u; 4D at equal time t = 1/2."""
    s = (np.arange(N, dtype=np.float64) + 1.0) / (N + 1.0)
    if d == 2:
        return np.stack([s, 1.0 - s])
    t = np.full(N, 0.5)
    return np.stack([t, (s - 0.5) * 0.5, np.zeros(N), np.zeros(N)])


def perm_coords_2d(perm) -> np.ndarray:
    """Light-cone coordinates of a 2D order: element a at ((a+1)/(N+1), (perm[a]+1)/(N+1))."""
    perm = np.asarray(perm, dtype=np.float64)
    N = perm.size
    a = (np.arange(N, dtype=np.float64) + 1.0) / (N + 1.0)
    return np.stack([a, (perm + 1.0) / (N + 1.0)])


def _philox_block(master: int, tag: int, ctr: int) -> np.ndarray:
    """Four uint64 words of Philox4x64-10 at counter (ctr,0,0,0), key (master, tag).
    numpy's generator advances its counter before each block, hence ctr-1."""
    g = np.random.Philox(key=[master & (U64 - 1), tag], counter=(ctr - 1) % 2**256)
    return g.random_raw(4)


def ensemble_plan(nsets: int = 512, master_seed: int = 4, n_lo: int = 256,
                  n_hi: int = 4096):
    """Per set s: seed = r0, N = n_lo + floor(r1 (n_hi-n_lo+1) / 2^64),
    d = 2 + 2 (r2 >> 63), with (r0,r1,r2,r3) = Philox(ctr=(s,0,0,0), key=(master, 3))."""
    span = n_hi - n_lo + 1
    plan = []
    for s in range(nsets):
        r = [int(x) for x in _philox_block(master_seed, 3, s)]
        N = n_lo + (r[1] * span >> 64)
        d = 2 + 2 * (r[2] >> 63)
        plan.append((d, N, r[0]))
    return plan


def request_plan(nreq: int = 10000, master_seed: int = 5, n_lo: int = 512,
                 n_hi: int = 32768, rate_per_s: float = 1000.0):
    """Per request q: seed = r0; N = floor(exp(ln n_lo + U ln(n_hi/n_lo))) clamped,
    U = (r1>>11) 2^-53; d = 2 + 2 (r2 >> 63); arrival gaps -ln(1-U')/rate with
    U' = (r3>>11) 2^-53.  Returns a list of (arrival_s, d, N, seed)."""
    out = []
    t = 0.0
    lo, hi = math.log(n_lo), math.log(n_hi / n_lo)
    for q in range(nreq):
        r = [int(x) for x in _philox_block(master_seed, 4, q)]
        U = (r[1] >> 11) * 2.0**-53
        N = int(math.floor(math.exp(lo + U * hi)))
        N = min(max(N, n_lo), n_hi)
        d = 2 + 2 * (r[2] >> 63)
        U2 = (r[3] >> 11) * 2.0**-53
        t += -math.log1p(-U2) / rate_per_s
        out.append((t, d, N, r[0]))
    return out


# The five workloads, with the seeds used everywhere.
WORKLOADS = {
    "2d_1024": dict(d=2, N=1024, seed=1),
    "4d_16384": dict(d=4, N=16384, seed=2),
    "2d_131072": dict(d=2, N=131072, seed=3),
}
