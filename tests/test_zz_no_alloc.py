"""vadx_top_k_noalloc (the ranking entry point that allocates nothing: its
scratch is a fixed device array) against vadx_top_k through the C ABI: two
calls in a row, the second with a smaller input, bit-identical indices and
scores; inputs above its stated maximum are rejected with a clear error."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _noalloc(ctx, score, k):
    import torch

    from paper_2311_13337_amd import vadx
    L = vadx.lib()
    f = L.vadx_top_k_noalloc
    f.restype = C.c_int
    f.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_int32, C.c_void_p, C.c_void_p]
    idx = torch.empty(max(k, 1), dtype=torch.int64, device="cuda")
    val = torch.empty(max(k, 1), dtype=torch.float32, device="cuda")
    st = f(ctx.h, C.c_void_p(score.data_ptr()), score.numel(), k, C.c_void_p(idx.data_ptr()),
           C.c_void_p(val.data_ptr()))
    return st, idx[:k].cpu().numpy(), val[:k].cpu().numpy()


def test_top_k_noalloc_matches_top_k():
    import torch

    from paper_2311_13337_amd import vadx
    ctx = vadx.Context(0)
    rng = np.random.default_rng(5)
    for n, k in ((3_000_000, 1000), (70_001, 37)):          # second call smaller
        s = (rng.integers(-400, 400, n) * 0.125).astype(np.float32)   # many ties
        d = torch.from_numpy(s).cuda()
        st, idx, val = _noalloc(ctx, d, k)
        assert st == vadx.VADX_OK, vadx.lib().vadx_last_error(ctx.h)
        want_idx, want_val = ctx.vadx_top_k(d, k)
        assert np.array_equal(idx, want_idx.cpu().numpy())
        assert np.array_equal(val, want_val.cpu().numpy())
        order = np.lexsort((np.arange(n), -s.astype(np.float64)))[:k]
        assert np.array_equal(idx, order)
    # above the stated maximum (2^24 scores): a clear error, nothing written
    big = torch.zeros((1 << 24) + 1, dtype=torch.float32, device="cuda")
    st, _, _ = _noalloc(ctx, big, 3)
    assert st == vadx.VADX_E_UNSUPPORTED
    assert b"at most" in vadx.lib().vadx_last_error(ctx.h)
