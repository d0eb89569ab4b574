"""GPU test of hd_rank_noalloc, the ranking entry point that allocates
nothing (its scratch is the library's fixed device array): through the C
ABI, two calls in a row on the same device, the second with fewer rows and
items, each against hd_rank on the same scores (bit-exact: ids and scores);
sizes above the fixed scratch are refused with HD_EINVAL and leave the
array usable."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def scores(B, n, seed):
    import torch
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((B, n)).astype(np.float32)
    x[:, ::7] = np.round(x[:, ::7], 1)  # ties, broken toward the lower id
    return torch.from_numpy(x).to(torch.device("cuda:0"))


def test_noalloc_matches_rank_twice():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1807_08692_amd import hd
    L = hd.lib()
    ctx = hd.Context(0)
    try:
        for B, n, K, seed in ((200, 300_000, 100, 1), (7, 5_003, 50, 2)):
            x = scores(B, n, seed)
            assert L.hd_rank_noalloc_scratch_bytes(B, n, K) <= 64 << 20
            ri, rs = ctx.rank(x, K)
            ni = torch.full((B, K), -1, dtype=torch.int32, device=x.device)
            ns = torch.full((B, K), np.nan, dtype=torch.float32, device=x.device)
            code = L.hd_rank_noalloc(ctx._h, B, n, ctypes.c_void_p(x.data_ptr()), n, K,
                                     ctypes.c_void_p(ni.data_ptr()), ctypes.c_void_p(ns.data_ptr()), None)
            assert code == hd.HD_OK, hd.last_error()
            torch.cuda.synchronize()
            assert torch.equal(ni, ri) and torch.equal(ns, rs), (B, n)
            # the selection itself: the K largest, equal scores to the lower id
            xc = x.cpu().numpy()
            for b in (0, B - 1):
                order = np.lexsort((np.arange(n), -xc[b]))[:K]
                assert np.array_equal(ni[b].cpu().numpy(), order)
        # a size above the fixed scratch is refused, and the next call works
        big = L.hd_rank_noalloc(ctx._h, 1024, 1_000_000, ctypes.c_void_p(x.data_ptr()), 1_000_000, 10,
                                ctypes.c_void_p(ni.data_ptr()), None, None)
        assert big == hd.HD_EINVAL and "scratch" in hd.last_error()
        ids, sc = ctx.rank_noalloc(x, 5)
        ri, rs = ctx.rank(x, 5)
        torch.cuda.synchronize()
        assert torch.equal(ids, ri) and torch.equal(sc, rs)
    finally:
        ctx.close()
