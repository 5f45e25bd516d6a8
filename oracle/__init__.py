"""CPU oracle for the causal-set interval-abundance path.

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only ``tests/``, ``__graft_entry__.smoke``
and the ``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares
no code with the GPU library (``paper_1709_03013_amd``) and neither imports the
other.

Two tiers, both written from the paper's definitions (arXiv:1709.03013):

* ``cs_oracle.c`` (plain C, OpenMP, ``-ffp-contract=off``): Philox4x64-10
  from its published definition, sprinkling and time sort (Sec. 2.1-2.2), the
  timelike relation (Sec. 1.1), the packed symmetric matrix (Sec. 2.2,
  Sec. 3.2), the triple-loop interval count of Sec. 4.1 (tier 1), the masked
  AND + popcount count of Fig. 2 / Alg. 5 over the bitset (tier 2), the
  3-chain identity and the BD action (Eq. 4; 4D weights are a reading), the
  smeared action (Eq. 5), and the (1+1) de Sitter slab of Sec. 6.1 (Eq. 9):
  sprinkle uniform in w = tan(eta) and in angle, and its relation.
* ``brute.py``: pure-Python brute force for tiny sets, used to pin the C code.

Every function here has pins in ``tests/test_oracle_*.py``.  The 4D action is
a reading (the paper prints only the 2D one, Eq. 4): its weights and index
convention are pinned by the identities Eq. 4's own weights satisfy in 2D
(weights summing to 0, a chain giving N - 1, the vanishing squared-proper-time
moment) and by hand-counted orders; its prefactor 4/sqrt(6) is "parity
unpinned" (nothing in the paper fixes it).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cs_oracle.c")
_BUILD = os.path.join(_HERE, "_build")
_LIB = os.path.join(_BUILD, "libcs_oracle.so")

_u64p = ctypes.POINTER(ctypes.c_uint64)
_i64p = ctypes.POINTER(ctypes.c_int64)
_dp = ctypes.POINTER(ctypes.c_double)


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc into ``oracle/_build/libcs_oracle.so``."""
    os.makedirs(_BUILD, exist_ok=True)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp",
               "-ffp-contract=off", "-fno-fast-math", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        L.orc_philox4x64_10.argtypes = [_u64p, _u64p, _u64p]
        L.orc_philox4x64_10.restype = None
        L.orc_sprinkle.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_uint64, _dp, _i64p]
        L.orc_sprinkle.restype = ctypes.c_int64
        L.orc_related.argtypes = [ctypes.c_int, _dp, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64]
        L.orc_related.restype = ctypes.c_int
        L.orc_row_words.argtypes = [ctypes.c_int64]
        L.orc_row_words.restype = ctypes.c_int64
        L.orc_link.argtypes = [ctypes.c_int, _dp, ctypes.c_int64, _u64p, ctypes.c_int64]
        L.orc_link.restype = None
        L.orc_count_coords.argtypes = [ctypes.c_int, _dp, ctypes.c_int64, ctypes.c_int64,
                                       ctypes.c_int64, ctypes.c_int64, _u64p, _u64p, _u64p]
        L.orc_count_coords.restype = None
        L.orc_interval_size.argtypes = [_u64p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64]
        L.orc_interval_size.restype = ctypes.c_uint64
        L.orc_count_bits.argtypes = [_u64p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                     ctypes.c_int64, ctypes.c_int64, _u64p, _u64p, _u64p,
                                     ctypes.c_int]
        L.orc_count_bits.restype = None
        L.orc_three_chains.argtypes = [_u64p, ctypes.c_int64, ctypes.c_int64]
        L.orc_three_chains.restype = ctypes.c_uint64
        L.orc_bd_action.argtypes = [ctypes.c_int, ctypes.c_int64, _u64p]
        L.orc_bd_action.restype = ctypes.c_double
        L.orc_smeared_action.argtypes = [ctypes.c_int64, _u64p, ctypes.c_int64, ctypes.c_double]
        L.orc_smeared_action.restype = ctypes.c_double
        L.orc_sprinkle_desitter.argtypes = [ctypes.c_int64, ctypes.c_uint64, ctypes.c_double, _dp, _i64p]
        L.orc_sprinkle_desitter.restype = ctypes.c_int64
        L.orc_related_desitter.argtypes = [_dp, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64]
        L.orc_related_desitter.restype = ctypes.c_int
        L.orc_link_desitter.argtypes = [_dp, ctypes.c_int64, _u64p, ctypes.c_int64]
        L.orc_link_desitter.restype = None
        L.orc_num_threads.argtypes = []
        L.orc_num_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a: np.ndarray, t):
    return a.ctypes.data_as(t)


def philox4x64_10(ctr, key) -> np.ndarray:
    """One Philox4x64-10 block: 4 uint64 outputs for a 4-word counter and 2-word key."""
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint64).reshape(4))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint64).reshape(2))
    out = np.zeros(4, dtype=np.uint64)
    lib().orc_philox4x64_10(_p(c, _u64p), _p(k, _u64p), _p(out, _u64p))
    return out


def row_words(N: int) -> int:
    """Words per packed row: ceil(N/64) rounded up to a multiple of 4 (256-bit rows)."""
    return int(lib().orc_row_words(N))


def sprinkle(d: int, N: int, seed: int):
    """Sorted coordinates (d x N float64, SoA), generation index of each
    sorted element, and the number of Philox candidates drawn."""
    coords = np.zeros((d, max(N, 0)), dtype=np.float64)
    orig = np.zeros(max(N, 0), dtype=np.int64)
    drawn = lib().orc_sprinkle(d, N, seed & (2**64 - 1), _p(coords, _dp), _p(orig, _i64p))
    if drawn < 0:
        raise ValueError("bad sprinkle arguments")
    return coords, orig, int(drawn)


def related(d: int, coords: np.ndarray, i: int, j: int) -> bool:
    c = np.ascontiguousarray(coords, dtype=np.float64)
    return bool(lib().orc_related(d, _p(c, _dp), c.shape[1], i, j))


def link(d: int, coords: np.ndarray) -> np.ndarray:
    """Packed symmetric matrix, shape (N, W) uint64."""
    c = np.ascontiguousarray(coords, dtype=np.float64)
    N = c.shape[1]
    W = row_words(N)
    bits = np.zeros((N, W), dtype=np.uint64)
    if N:
        lib().orc_link(d, _p(c, _dp), N, _p(bits, _u64p), W)
    return bits


def count_coords(d: int, coords: np.ndarray, nbins: int | None = None,
                 rows: tuple[int, int] | None = None):
    """Tier 1 (triple loop on coordinates).  Returns (hist[nbins], R, summ)."""
    c = np.ascontiguousarray(coords, dtype=np.float64)
    N = c.shape[1]
    nb = nbins if nbins is not None else max(N - 1, 1)
    lo, hi = rows if rows is not None else (0, N)
    hist = np.zeros(nb, dtype=np.uint64)
    R = ctypes.c_uint64(0)
    s = ctypes.c_uint64(0)
    lib().orc_count_coords(d, _p(c, _dp), N, lo, hi, nb, _p(hist, _u64p),
                           ctypes.byref(R), ctypes.byref(s))
    return hist, int(R.value), int(s.value)


def count_bits(bits: np.ndarray, N: int, nbins: int | None = None,
               rows: tuple[int, int] | None = None, nthreads: int = 0):
    """Tier 2 (masked AND + popcount over the packed rows).  Returns (hist, R, summ)."""
    b = np.ascontiguousarray(bits, dtype=np.uint64)
    W = b.shape[1] if b.ndim == 2 else row_words(N)
    nb = nbins if nbins is not None else max(N - 1, 1)
    lo, hi = rows if rows is not None else (0, N)
    hist = np.zeros(nb, dtype=np.uint64)
    R = ctypes.c_uint64(0)
    s = ctypes.c_uint64(0)
    lib().orc_count_bits(_p(b, _u64p), N, W, lo, hi, nb, _p(hist, _u64p),
                         ctypes.byref(R), ctypes.byref(s), nthreads)
    return hist, int(R.value), int(s.value)


def interval_size(bits: np.ndarray, i: int, j: int) -> int:
    b = np.ascontiguousarray(bits, dtype=np.uint64)
    return int(lib().orc_interval_size(_p(b, _u64p), b.shape[1], i, j))


def three_chains(bits: np.ndarray, N: int) -> int:
    b = np.ascontiguousarray(bits, dtype=np.uint64)
    return int(lib().orc_three_chains(_p(b, _u64p), N, b.shape[1]))


def bd_action(d: int, N: int, n) -> float:
    a = np.ascontiguousarray(np.asarray(n, dtype=np.uint64)[:4])
    if a.size < 4:
        a = np.concatenate([a, np.zeros(4 - a.size, dtype=np.uint64)])
    return float(lib().orc_bd_action(d, N, _p(a, _u64p)))


def smeared_action(N: int, hist, eps: float) -> float:
    """Eq. 5 from the full histogram hist[k] = N_k (k = 0..len-1)."""
    h = np.ascontiguousarray(np.asarray(hist, dtype=np.uint64))
    return float(lib().orc_smeared_action(N, _p(h, _u64p), h.size, eps))


def sprinkle_desitter(N: int, seed: int, eta0: float):
    """(1+1) de Sitter slab: sorted (w = tan eta, x, y) SoA, generation index,
    Philox blocks drawn.  w0 = tan(eta0) is rounded once by the host libm."""
    import math
    coords = np.zeros((3, max(N, 0)), dtype=np.float64)
    orig = np.zeros(max(N, 0), dtype=np.int64)
    drawn = lib().orc_sprinkle_desitter(N, seed & (2**64 - 1), math.tan(eta0), _p(coords, _dp), _p(orig, _i64p))
    if drawn < 0:
        raise ValueError("bad sprinkle arguments")
    return coords, orig, int(drawn)


def related_desitter(coords: np.ndarray, i: int, j: int) -> bool:
    c = np.ascontiguousarray(coords, dtype=np.float64)
    return bool(lib().orc_related_desitter(_p(c, _dp), c.shape[1], i, j))


def link_desitter(coords: np.ndarray) -> np.ndarray:
    c = np.ascontiguousarray(coords, dtype=np.float64)
    N = c.shape[1]
    W = row_words(N)
    bits = np.zeros((N, W), dtype=np.uint64)
    if N:
        lib().orc_link_desitter(_p(c, _dp), N, _p(bits, _u64p), W)
    return bits


def num_threads() -> int:
    return int(lib().orc_num_threads())


def causal_set(d: int, N: int, seed: int, nbins: int = 4):
    """The whole path for one sprinkled set: coords, bits, hist, R, summ, S."""
    coords, _, _ = sprinkle(d, N, seed)
    bits = link(d, coords)
    hist, R, s = count_bits(bits, N, nbins=nbins)
    S = bd_action(d, N, hist[:4])
    return coords, bits, hist, R, s, S
