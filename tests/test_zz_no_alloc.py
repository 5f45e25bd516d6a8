"""GPU: the count with the library's own workspace (cs_count_dev_static)
against the same count with a caller's workspace (cs_count_dev) and the
oracle, two calls in a row with the second on a smaller input, through the C
ABI."""
import sys

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_static_workspace_count_matches_caller_workspace():
    import torch

    import paper_1709_03013_amd as cs
    stream = torch.cuda.current_stream()
    ctx = cs.cs_create(0, 0, stream.cuda_stream)
    try:
        # the first call leaves 43-word rows in the array; the second, smaller
        # one must not see them
        for d, N, seed, kmax, path in [(2, 9000, 5, 40, 3), (4, 3000, 6, 3, 2), (2, 700, 7, 3, 1),
                                       (2, 500, 8, 3, 3)]:
            say("case static workspace d=%d N=%d kmax=%d path=%d" % (d, N, kmax, path))
            s = cs.cs_sprinkle(ctx, d, N, seed)
            try:
                cs.cs_link(ctx, s)
                bits = cs.cs_set_bitset_dev(s)
                W = cs.cs_row_words(N)
                a = torch.full((kmax + 3,), -1, dtype=torch.int64, device="cuda:0")
                b = torch.full((kmax + 3,), -1, dtype=torch.int64, device="cuda:0")
                ws = torch.empty(cs.cs_count_workspace_bytes(N, kmax) // 8, dtype=torch.int64,
                                 device="cuda:0")
                cs.cs_count_dev(bits, N, W, kmax, a.data_ptr(), ws.data_ptr(), path, stream.cuda_stream)
                cs.cs_count_dev_static(bits, N, W, kmax, b.data_ptr(), path, stream.cuda_stream)
                torch.cuda.synchronize()
                assert torch.equal(a, b), (a, b)
                oc, _, _ = oracle.sprinkle(d, N, seed)
                h, R, sm = oracle.count_bits(oracle.link(d, oc), N, nbins=kmax + 1)
                got = b.cpu().numpy().view(np.uint64)
                assert list(got[:kmax + 1]) == list(h) and got[kmax + 1] == R and got[kmax + 2] == sm
            finally:
                cs.cs_set_free(s)
        # a workspace beyond the array is refused before anything runs
        with pytest.raises(cs.CsError) as e:
            cs.cs_count_dev_static(1, 131072, cs.cs_row_words(131072), 300, 1, 3, None)
        assert e.value.status == 1
    finally:
        cs.cs_destroy(ctx)
