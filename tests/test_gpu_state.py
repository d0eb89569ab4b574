"""GPU checks of the context's state across rejected loader calls: a call
that fails its argument checks leaves what was loaded before untouched, so
the next query runs on it and gives the same results as before; an unload
(r = 0) leaves plain CG."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1807_08692_amd import workload as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fx = W.build_fixture(W.CONFIGS["n5k"], n_queries=8, prefer_gpu=False)
    ids, vals = [], []
    for q in fx.Q[:8]:
        i, v = O.observation(fx.V, q, fx.cfg.k_y)
        ids.append(i)
        vals.append(v)
    dev = torch.device("cuda:0")
    return fx, torch.from_numpy(np.stack(ids).astype(np.int32)).to(dev), \
        torch.from_numpy(np.stack(vals).astype(np.float32)).to(dev)


@pytest.mark.parametrize("dtype", ["f32", "bf16x2", "fp8"])
def test_rejected_load_eigs_keeps_state(setup, dtype):
    import torch
    from paper_1807_08692_amd import hd
    fx, ti, tv = setup
    kw = dict(alpha=0.99, tol=0.0, max_iter=6, k_y=fx.cfg.k_y, top_k=20, want_x=True)
    c = hd.Context(0)
    try:
        c.load_graph(fx.n, fx.rowptr, fx.col, fx.s)
        c.load_eigs(fx.U, fx.lam, dtype=dtype)
        before = c.query_batch(None, ti, tv, rank_r=-1, **kw)["x"].cpu().numpy()
        bad_lam = fx.lam.copy()
        bad_lam[3] = 1.5
        with pytest.raises(hd.HDError):
            c.load_eigs(fx.U, bad_lam, dtype="bf16")
        bad_U = fx.U.copy()
        bad_U[10, 2] = np.nan
        with pytest.raises(hd.HDError):
            c.load_eigs(bad_U, fx.lam, dtype="bf16x2")
        with pytest.raises(hd.HDError):
            c.load_eigs_fp8(np.full((fx.n, 4), 0x7F, np.uint8), np.ones(4, np.float32), fx.lam[:4])
        after = c.query_batch(None, ti, tv, rank_r=-1, **kw)["x"].cpu().numpy()
        torch.cuda.synchronize()
        assert np.array_equal(before, after)
        # unloading leaves plain CG: rank_r = -1 is then r = 0
        c.load_eigs(np.zeros((fx.n, 0), np.float32), np.zeros(0))
        plain = c.query_batch(None, ti, tv, rank_r=-1, **kw)["x"].cpu().numpy()
        plain0 = c.query_batch(None, ti, tv, rank_r=0, **kw)["x"].cpu().numpy()
        assert np.array_equal(plain, plain0)
        with pytest.raises(hd.HDError):
            c.query_batch(None, ti, tv, rank_r=5, **kw)
    finally:
        c.close()


def test_rejected_descriptors_keep_state(setup):
    import torch
    from paper_1807_08692_amd import hd
    fx, _, _ = setup
    c = hd.Context(0)
    try:
        c.load_graph(fx.n, fx.rowptr, fx.col, fx.s)
        c.load_descriptors(fx.V, dtype="bf16")
        q = torch.from_numpy(fx.Q[:4]).to(torch.device("cuda:0"))
        before = c.query_batch(q, max_iter=3, rank_r=0, k_y=fx.cfg.k_y, top_k=10)["rank_ids"].cpu().numpy()
        bad = fx.V.copy()
        bad[7, 0] = np.inf
        with pytest.raises(hd.HDError):
            c.load_descriptors(bad, dtype="fp8")
        after = c.query_batch(q, max_iter=3, rank_r=0, k_y=fx.cfg.k_y, top_k=10)["rank_ids"].cpu().numpy()
        assert np.array_equal(before, after)
    finally:
        c.close()
