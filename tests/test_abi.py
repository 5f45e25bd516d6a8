"""The C-ABI library loads and exports every symbol include/cs.h declares
(CPU only: no compute calls), and its argument checks run before any device
work."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cs.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(cs_[a-z_]+)\s*\(", src)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    import paper_1709_03013_amd as p
    return p


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ["cs_create", "cs_destroy", "cs_last_error", "cs_sprinkle", "cs_link",
                 "cs_interval_abundances", "cs_bd_action", "cs_set_from_bitset", "cs_get_bitset",
                 "cs_get_coords", "cs_link_dev", "cs_count_dev", "cs_batch_run",
                 "cs_queue_submit", "cs_queue_poll", "cs_queue_drain"]:
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    so = lib._binding.LIB_PATH
    out = subprocess.run(["nm", "-D", "--defined-only", so], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT (cs_[a-z_]+)\b", out))
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing


def test_binding_covers_every_declared_symbol(lib):
    assert sorted(lib.exported_symbols()) == declared_functions()
    L = lib.lib()
    for n in declared_functions():
        assert hasattr(L, n)


def test_row_words(lib):
    assert lib.cs_row_words(0) == 0
    assert lib.cs_row_words(1) == 4
    assert lib.cs_row_words(64) == 4
    assert lib.cs_row_words(257) == 8
    assert lib.cs_row_words(1024) == 16
    assert lib.cs_row_words(131072) == 2048


def test_argument_errors_need_no_device(lib):
    with pytest.raises(lib.CsError) as e:
        lib.cs_link_dev(3, 10, 0, 0, 4, None, 0, None)
    assert e.value.status == lib._binding.CS_EINVAL
    with pytest.raises(lib.CsError) as e:
        lib.cs_link_dev(2, 100, 1, 1, 3, 1, 1 << 20, None)   # stride too small
    assert e.value.status == lib._binding.CS_EINVAL
    need = lib.cs_link_workspace_bytes(2, 100)
    assert need == 2 * 2112                               # two blocks of 64 labels
    assert lib.cs_link_workspace_bytes(4, 100) == 0
    with pytest.raises(lib.CsError) as e:
        lib.cs_link_dev(2, 100, 1, 1, 4, None, 0, None)      # 2D without its tables
    assert e.value.status == lib._binding.CS_EINVAL
    with pytest.raises(lib.CsError) as e:
        lib.cs_link_dev(2, 100, 1, 1, 4, 1, need - 8, None)  # workspace too small
    assert e.value.status == lib._binding.CS_EINVAL
    with pytest.raises(lib.CsError) as e:
        lib.cs_count_dev(1, 100, 4, 2, 1, 1, 0, None)   # kmax < 3
    assert e.value.status == lib._binding.CS_EINVAL
    with pytest.raises(lib.CsError) as e:
        lib.cs_count_dev(1, 100, 4, 3, 1, 1, 7, None)   # bad path
    assert e.value.status == lib._binding.CS_EINVAL
    assert lib.cs_count_workspace_bytes(1000, 3) == 4 * 6 * 8


def test_static_workspace_count_refuses_before_any_device_work(lib):
    """cs_count_dev_static checks its arguments and the size of the library's
    array (CS_COUNT_STATIC_WORDS words) before touching a device."""
    EINVAL = lib._binding.CS_EINVAL
    W = lib.cs_row_words(131072)
    cases = [(131072, W, 300, 3),      # 512 row blocks x 303 words > 131072
             (2 ** 20, lib.cs_row_words(2 ** 20), 30, 2),
             (100, 4, 2, 1),           # kmax < 3
             (100, 4, 3, 9),           # bad path
             (100, 2, 3, 1),           # stride below W
             (-1, 4, 3, 1)]
    for N, stride, kmax, path in cases:
        with pytest.raises(lib.CsError) as e:
            lib.cs_count_dev_static(1, N, stride, kmax, 1, path, None)
        assert e.value.status == EINVAL, (N, stride, kmax, path)
    assert lib._binding.COUNT_STATIC_WORDS == 131072
    # the largest full histogram that fits at N = 2^17: 512 * (253 + 3) words
    assert lib.cs_count_workspace_bytes(131072, 253) // 8 <= lib._binding.COUNT_STATIC_WORDS
    assert lib.cs_count_workspace_bytes(131072, 254) // 8 > lib._binding.COUNT_STATIC_WORDS


def test_local_count_argument_errors_need_no_device(lib):
    EINVAL = lib._binding.CS_EINVAL
    ws = lambda N: 64 * max((N + 63) // 64, 1)
    cases = [(-1, 4, 1, 1, 10**6),                 # N < 0
             (100, 4, 0, 1, 10**6), (100, 4, 1, 0, 10**6),   # NULL stats / work
             (100, 3, 1, 1, 10**6), (100, 6, 1, 1, 10**6),   # stride below W, not a multiple of 4
             (100, 4, 1, 1, ws(100) - 8)]          # workspace below the size
    for N, stride, stats, work, wb in cases:
        with pytest.raises(lib.CsError) as e:
            lib.cs_count_local_dev(1, N, stride, stats, work, wb, None)
        assert e.value.status == EINVAL, (N, stride, stats, work, wb)
    assert lib.cs_count_local_workspace_bytes(0) == 64
    assert lib.cs_count_local_workspace_bytes(131072) == 64 * 2048
    assert lib.cs_count_local_workspace_bytes(-1) == 0


def test_no_device_is_an_error_not_a_fallback(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(lib.CsError) as e:
        lib.cs_create(0)
    assert e.value.status in (lib._binding.CS_EDEVICE, lib._binding.CS_EINVAL)


def test_struct_layouts(lib):
    import ctypes
    b = lib._binding
    assert ctypes.sizeof(b.cs_batch_info) == 6 * 4 + 2 * 8
    assert ctypes.sizeof(b.cs_req) == 24
    assert ctypes.sizeof(b.cs_result) == 4 * 8 + 8 + 8 + 8 + 8
