"""ctypes binding of ``libcs_gfx950.so`` (include/cs.h).

Argument marshalling only: every step of the path runs inside the library's
HIP kernels.  Functions keep the C names; failures raise ``CsError`` with the
library's message.  The library must have been built (``build.py``); there is
no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcs_gfx950.so")

CS_OK, CS_EINVAL, CS_ENOMEM, CS_EDEVICE, CS_EBUSY, CS_EUNSUPPORTED = range(6)
PATH_AUTO, PATH_POP, PATH_MFMA, PATH_MFMA_FP4, PATH_LOCAL = 0, 1, 2, 3, 4
ROW_BLOCK = 256
KMAX_MAX = 16777213
STATUS_NAMES = {0: "CS_OK", 1: "CS_EINVAL", 2: "CS_ENOMEM", 3: "CS_EDEVICE",
                4: "CS_EBUSY", 5: "CS_EUNSUPPORTED"}


class CsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


class cs_req(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("N", ctypes.c_int64), ("seed", ctypes.c_uint64)]


class cs_result(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint64 * 4), ("R", ctypes.c_uint64), ("summ", ctypes.c_uint64),
                ("S", ctypes.c_double), ("status", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {"n": [int(x) for x in self.n], "R": int(self.R), "summ": int(self.summ),
                "S": float(self.S), "status": int(self.status)}


class cs_batch_info(ctypes.Structure):
    _fields_ = [("sets_pop", ctypes.c_int32), ("sets_mfma256", ctypes.c_int32),
                ("sets_mfma128", ctypes.c_int32), ("grid_pop", ctypes.c_int32),
                ("grid_mfma256", ctypes.c_int32), ("grid_mfma128", ctypes.c_int32),
                ("count_ms_untuned", ctypes.c_double), ("count_ms_tuned", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_vp = ctypes.c_void_p
_u64p = ctypes.POINTER(ctypes.c_uint64)
_i64p = ctypes.POINTER(ctypes.c_int64)
_dp = ctypes.POINTER(ctypes.c_double)

_SIGS = {
    "cs_row_words": (ctypes.c_int64, [ctypes.c_int64]),
    "cs_create": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_uint64, _vp]),
    "cs_destroy": (None, [_vp]),
    "cs_last_error": (ctypes.c_char_p, []),
    "cs_bytes_in_use": (ctypes.c_uint64, [_vp]),
    "cs_sprinkle": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int64, ctypes.c_uint64, ctypes.POINTER(_vp)]),
    "cs_set_from_coords": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int64, _dp, ctypes.POINTER(_vp)]),
    "cs_set_from_bitset": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int64, _vp, ctypes.c_int64,
                                          ctypes.c_int, ctypes.c_int, ctypes.POINTER(_vp)]),
    "cs_set_free": (None, [_vp]),
    "cs_set_info": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int), _i64p, _i64p,
                                   ctypes.POINTER(ctypes.c_int)]),
    "cs_get_coords": (ctypes.c_int, [_vp, _vp, _dp, _i64p]),
    "cs_sprinkle_desitter": (ctypes.c_int, [_vp, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double,
                                            ctypes.POINTER(_vp)]),
    "cs_set_manifold": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
    "cs_get_bitset": (ctypes.c_int, [_vp, _vp, _u64p]),
    "cs_set_bitset_dev": (_vp, [_vp]),
    "cs_set_count_path": (ctypes.c_int, [_vp]),
    "cs_link": (ctypes.c_int, [_vp, _vp]),
    "cs_interval_abundances": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _u64p, _u64p, _u64p, ctypes.c_int]),
    "cs_interval_abundances_rows": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _u64p, ctypes.c_int]),
    "cs_bd_action": (ctypes.c_int, [_vp, _vp, _dp]),
    "cs_smeared_action": (ctypes.c_int, [_vp, _vp, ctypes.c_double, _dp]),
    "cs_link_workspace_bytes": (ctypes.c_uint64, [ctypes.c_int, ctypes.c_int64]),
    "cs_link_dev": (ctypes.c_int, [ctypes.c_int, ctypes.c_int64, _vp, _vp, ctypes.c_int64, _vp,
                                   ctypes.c_uint64, _vp]),
    "cs_count_workspace_bytes": (ctypes.c_uint64, [ctypes.c_int64, ctypes.c_int]),
    "cs_count_dev": (ctypes.c_int, [_vp, ctypes.c_int64, ctypes.c_int64, ctypes.c_int, _vp, _vp,
                                    ctypes.c_int, _vp]),
    "cs_count_dev_static": (ctypes.c_int, [_vp, ctypes.c_int64, ctypes.c_int64, ctypes.c_int, _vp,
                                           ctypes.c_int, _vp]),
    "cs_local_abundances": (ctypes.c_int, [_vp, _vp, _u64p, _u64p]),
    "cs_count_local_workspace_bytes": (ctypes.c_uint64, [ctypes.c_int64]),
    "cs_count_local_dev": (ctypes.c_int, [_vp, ctypes.c_int64, ctypes.c_int64, _vp, _vp,
                                          ctypes.c_uint64, _vp]),
    "cs_batch_run": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.POINTER(cs_req), ctypes.POINTER(cs_result)]),
    "cs_batch_last_info": (ctypes.c_int, [_vp, ctypes.POINTER(cs_batch_info)]),
    "cs_queue_start": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_uint64]),
    "cs_queue_submit": (ctypes.c_int, [_vp, ctypes.POINTER(cs_req), _u64p]),
    "cs_queue_poll": (ctypes.c_int, [_vp, ctypes.c_uint64, ctypes.POINTER(cs_result), _dp]),
    "cs_queue_next": (ctypes.c_int, [_vp, ctypes.c_double, _u64p, ctypes.POINTER(cs_result), _dp]),
    "cs_queue_drain": (ctypes.c_int, [_vp]),
    "cs_queue_stop": (ctypes.c_int, [_vp]),
}

_lib = None


def _bind_one_hip_runtime():
    """Import torch first when it is installed: it loads its own HIP runtime
    (soname libamdhip64.so.7), and the library then binds to that same copy.
    Two HIP runtimes in one process cannot share the device."""
    try:
        import torch  # noqa: F401
    except ImportError:
        pass


def lib() -> ctypes.CDLL:
    """Load the built library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        _bind_one_hip_runtime()
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libcs_gfx950.so is not built: run python -m paper_1709_03013_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGS)


def _check(rc: int):
    if rc != CS_OK:
        raise CsError(rc, lib().cs_last_error().decode(errors="replace"))


def _ptr(a: np.ndarray, t):
    return a.ctypes.data_as(t)


# ------------------------------------------------------------------ C names
def cs_row_words(N: int) -> int:
    return int(lib().cs_row_words(N))


def cs_create(device: int = 0, hbm_budget_bytes: int = 0, hip_stream: int | None = None) -> int:
    h = _vp()
    _check(lib().cs_create(ctypes.byref(h), device, hbm_budget_bytes, hip_stream))
    return h.value


def cs_destroy(ctx: int) -> None:
    lib().cs_destroy(ctx)


def cs_bytes_in_use(ctx: int) -> int:
    return int(lib().cs_bytes_in_use(ctx))


def cs_sprinkle(ctx: int, d: int, N: int, seed: int) -> int:
    h = _vp()
    _check(lib().cs_sprinkle(ctx, d, N, seed % 2**64, ctypes.byref(h)))
    return h.value


CS_MANIFOLD_DIAMOND = 0
CS_MANIFOLD_DESITTER = 1


def cs_sprinkle_desitter(ctx: int, N: int, seed: int, eta0: float) -> int:
    h = _vp()
    _check(lib().cs_sprinkle_desitter(ctx, N, seed % 2**64, float(eta0), ctypes.byref(h)))
    return h.value


def cs_set_from_coords(ctx: int, d: int, coords: np.ndarray) -> int:
    c = np.ascontiguousarray(coords, dtype=np.float64)
    N = c.shape[1] if c.ndim == 2 else 0
    h = _vp()
    _check(lib().cs_set_from_coords(ctx, d, N, _ptr(c, _dp), ctypes.byref(h)))
    return h.value


def cs_set_from_bitset(ctx: int, d: int, N: int, rows, stride_words: int | None = None,
                       on_device: bool = False, validate: bool = True) -> int:
    h = _vp()
    if on_device:
        ptr = int(rows)
        stride = int(stride_words)
    else:
        r = np.ascontiguousarray(rows, dtype=np.uint64)
        stride = r.shape[1] if r.ndim == 2 else cs_row_words(N)
        ptr = r.ctypes.data
    _check(lib().cs_set_from_bitset(ctx, d, N, ptr, stride, 1 if on_device else 0,
                                    1 if validate else 0, ctypes.byref(h)))
    return h.value


def cs_set_free(s: int) -> None:
    lib().cs_set_free(s)


def cs_set_info(s: int):
    d = ctypes.c_int()
    N = ctypes.c_int64()
    W = ctypes.c_int64()
    linked = ctypes.c_int()
    _check(lib().cs_set_info(s, ctypes.byref(d), ctypes.byref(N), ctypes.byref(W), ctypes.byref(linked)))
    return d.value, N.value, W.value, bool(linked.value)


def cs_set_manifold(s: int):
    m = ctypes.c_int()
    rows = ctypes.c_int()
    _check(lib().cs_set_manifold(s, ctypes.byref(m), ctypes.byref(rows)))
    return m.value, rows.value


def cs_get_coords(ctx: int, s: int):
    _, N, _, _ = cs_set_info(s)
    _, rows = cs_set_manifold(s)
    coords = np.zeros((rows, N), dtype=np.float64)
    orig = np.zeros(N, dtype=np.int64)
    _check(lib().cs_get_coords(ctx, s, _ptr(coords, _dp), _ptr(orig, _i64p)))
    return coords, orig


def cs_get_bitset(ctx: int, s: int) -> np.ndarray:
    _, N, W, _ = cs_set_info(s)
    rows = np.zeros((N, W), dtype=np.uint64)
    _check(lib().cs_get_bitset(ctx, s, _ptr(rows, _u64p)))
    return rows


def cs_set_bitset_dev(s: int) -> int:
    return int(lib().cs_set_bitset_dev(s) or 0)


def cs_set_count_path(s: int) -> int:
    return int(lib().cs_set_count_path(s))


def cs_link(ctx: int, s: int) -> None:
    _check(lib().cs_link(ctx, s))


def cs_interval_abundances(ctx: int, s: int, kmax: int = 3, path: int = PATH_AUTO):
    out = np.zeros(kmax + 1, dtype=np.uint64)
    R = ctypes.c_uint64()
    sm = ctypes.c_uint64()
    _check(lib().cs_interval_abundances(ctx, s, kmax, _ptr(out, _u64p), ctypes.byref(R),
                                        ctypes.byref(sm), path))
    return out, int(R.value), int(sm.value)


def cs_interval_abundances_rows(ctx: int, s: int, kmax: int = 3, path: int = PATH_AUTO) -> np.ndarray:
    _, N, _, _ = cs_set_info(s)
    nrb = (N + ROW_BLOCK - 1) // ROW_BLOCK
    blocks = np.zeros((nrb, kmax + 3), dtype=np.uint64)
    _check(lib().cs_interval_abundances_rows(ctx, s, kmax, _ptr(blocks, _u64p), path))
    return blocks


def cs_local_abundances(ctx: int, s: int, blocks: bool = False):
    """(N_0..N_3 as uint64[4], R, pairs continued from HBM) by the saturating
    count; with blocks=True also the per-64-label-block breakdown,
    uint64[ceil(N/64), 5]."""
    out = np.zeros(6, dtype=np.uint64)
    blk = None
    if blocks:
        _, N, _, _ = cs_set_info(s)
        blk = np.zeros((max((N + 63) // 64, 1), 5), dtype=np.uint64)
    _check(lib().cs_local_abundances(ctx, s, _ptr(out, _u64p), _ptr(blk, _u64p) if blocks else None))
    res = (out[:4].copy(), int(out[4]), int(out[5]))
    return res + (blk,) if blocks else res


def cs_count_local_workspace_bytes(N: int) -> int:
    return int(lib().cs_count_local_workspace_bytes(N))


def cs_count_local_dev(bits_dev: int, N: int, stride_words: int, stats_dev: int, work_dev: int,
                       work_bytes: int, hip_stream: int | None):
    _check(lib().cs_count_local_dev(bits_dev, N, stride_words, stats_dev, work_dev, work_bytes,
                                    hip_stream))


def cs_bd_action(ctx: int, s: int) -> float:
    S = ctypes.c_double()
    _check(lib().cs_bd_action(ctx, s, ctypes.byref(S)))
    return S.value


def cs_smeared_action(ctx: int, s: int, eps: float) -> float:
    S = ctypes.c_double()
    _check(lib().cs_smeared_action(ctx, s, eps, ctypes.byref(S)))
    return S.value


def cs_link_workspace_bytes(d: int, N: int) -> int:
    return int(lib().cs_link_workspace_bytes(d, N))


def cs_link_dev(d: int, N: int, coords_dev: int, bits_dev: int, stride_words: int, work_dev: int | None,
                work_bytes: int, hip_stream: int | None):
    _check(lib().cs_link_dev(d, N, coords_dev, bits_dev, stride_words, work_dev, work_bytes, hip_stream))


def cs_count_workspace_bytes(N: int, kmax: int) -> int:
    return int(lib().cs_count_workspace_bytes(N, kmax))


def cs_count_dev(bits_dev: int, N: int, stride_words: int, kmax: int, stats_dev: int, work_dev: int,
                 path: int, hip_stream: int | None):
    _check(lib().cs_count_dev(bits_dev, N, stride_words, kmax, stats_dev, work_dev, path, hip_stream))


COUNT_STATIC_WORDS = 131072


def cs_count_dev_static(bits_dev: int, N: int, stride_words: int, kmax: int, stats_dev: int,
                        path: int, hip_stream: int | None):
    _check(lib().cs_count_dev_static(bits_dev, N, stride_words, kmax, stats_dev, path, hip_stream))


def make_reqs(plan):
    """plan: iterable of (d, N, seed)."""
    plan = list(plan)
    arr = (cs_req * max(len(plan), 1))()
    for k, (d, N, seed) in enumerate(plan):
        arr[k].d = d
        arr[k].N = N
        arr[k].seed = seed % 2**64
    return arr


class BatchCall:
    """The marshalled arguments of cs_batch_run for one list of (d, N, seed):
    the request and result arrays are built once, so repeated calls pass
    straight to the library (run), and the results are converted on demand
    (results)."""

    def __init__(self, plan):
        plan = list(plan)
        self.n = len(plan)
        self.reqs = make_reqs(plan)
        self.out = (cs_result * max(self.n, 1))()

    def run(self, ctx: int) -> None:
        _check(lib().cs_batch_run(ctx, self.n, self.reqs, self.out))

    def results(self):
        return [self.out[k].as_dict() for k in range(self.n)]


def cs_batch_run(ctx: int, plan):
    call = BatchCall(plan)
    call.run(ctx)
    return call.results()


def cs_batch_last_info(ctx: int) -> dict:
    info = cs_batch_info()
    _check(lib().cs_batch_last_info(ctx, ctypes.byref(info)))
    return info.as_dict()


def cs_queue_start(ctx: int, slots: int = 4, resident_budget: int = 0):
    _check(lib().cs_queue_start(ctx, slots, resident_budget))


def cs_queue_submit(ctx: int, d: int, N: int, seed: int) -> int:
    r = cs_req(d=d, reserved=0, N=N, seed=seed % 2**64)
    t = ctypes.c_uint64()
    _check(lib().cs_queue_submit(ctx, ctypes.byref(r), ctypes.byref(t)))
    return int(t.value)


def cs_queue_poll(ctx: int, ticket: int):
    """None while busy, else (result dict, (wait_s, run_s, total_s))."""
    out = cs_result()
    tm = (ctypes.c_double * 3)()
    rc = lib().cs_queue_poll(ctx, ticket, ctypes.byref(out), tm)
    if rc == CS_EBUSY:
        return None
    _check(rc)
    return out.as_dict(), (tm[0], tm[1], tm[2])


def cs_queue_next(ctx: int, timeout_s: float = 0.0):
    """None if nothing finished within timeout_s, else (ticket, result dict,
    (wait_s, run_s, total_s)) of the next finished request."""
    t = ctypes.c_uint64()
    out = cs_result()
    tm = (ctypes.c_double * 3)()
    rc = lib().cs_queue_next(ctx, float(timeout_s), ctypes.byref(t), ctypes.byref(out), tm)
    if rc == CS_EBUSY:
        return None
    _check(rc)
    return int(t.value), out.as_dict(), (tm[0], tm[1], tm[2])


def cs_queue_drain(ctx: int):
    _check(lib().cs_queue_drain(ctx))


def cs_queue_stop(ctx: int):
    _check(lib().cs_queue_stop(ctx))
