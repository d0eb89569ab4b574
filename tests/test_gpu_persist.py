"""GPU tests of the persistent CG kernel (hd_set_persistent): every CG
iteration of a narrow batch in one kernel, solver vectors as wide as the
batch rounded up to a power of two.

Against the FP64 oracle run on the GPU's own y for the GPU's per-column
iteration count: x to relative L2 error 1e-4 and the ranking exactly (the
oracle's sort of the GPU's x), for plain CG and fp32 U1, on the 5,000-item
workload (batches of 1, 3 and 16, CG to relative residual 1e-6) and on a
ragged random graph (1237 items, r = 37, widths 8, 16, 64). The iteration
counts and statuses match the multi-kernel path's; a HIP-graph plan replays
the persistent batch bit for bit; a wait bound of one polling round ends the
kernel early and the call reports it, after which the next call runs
normally."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1807_08692_amd import workload as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def fx():
    return W.build_fixture(W.CONFIGS["n5k"], n_queries=40, prefer_gpu=False)


@pytest.fixture(scope="module")
def g64(fx):
    return O.Graph64.from_csr(fx.n, fx.rowptr, fx.col, fx.s)


def oracle_y(fx, qs):
    ids, vals = [], []
    for q in qs:
        i, v = O.observation(fx.V, q, fx.cfg.k_y)
        ids.append(i)
        vals.append(v)
    return np.stack(ids).astype(np.int32), np.stack(vals).astype(np.float32)


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("B", [1, 3, 16])
@pytest.mark.parametrize("r", [0, 50])
def test_persistent_parity_workload(fx, g64, torch_dev, B, r):
    import torch
    from paper_1807_08692_amd import hd
    c = hd.Context(0)
    try:
        c.load_graph(fx.n, fx.rowptr, fx.col, fx.s)
        c.load_eigs(fx.U, fx.lam, dtype="f32")
        c.load_descriptors(fx.V)
        q = torch.from_numpy(fx.Q[:B]).to(torch_dev)
        kw = dict(alpha=0.99, max_iter=20, tol=1e-6, rank_r=r, k_y=fx.cfg.k_y, top_k=50, want_x=True,
                  want_y=True)
        eager = c.query_batch(q, **kw)
        torch.cuda.synchronize()
        c.set_persistent(1)
        pers = c.query_batch(q, **kw)
        torch.cuda.synchronize()
        assert np.array_equal(pers["y_ids"].cpu().numpy(), eager["y_ids"].cpu().numpy())
        assert np.array_equal(pers["status"], eager["status"])
        assert np.all(np.abs(pers["iters"] - eager["iters"]) <= 1)
        U = fx.U if r else None
        for b in range(B):
            yi = pers["y_ids"][b].cpu().numpy()
            yv = pers["y_val"][b].cpu().numpy()
            xo, *_ = O.iterate(g64, U, fx.lam if r else None, 0.99, yi, yv, int(pers["iters"][b]), 0.0)
            x = pers["x"][b].double().cpu().numpy()
            assert rel(x, xo) <= 1e-4, (B, r, b, rel(x, xo))
            oid, _ = O.rank(x, 50)
            assert np.array_equal(pers["rank_ids"][b].cpu().numpy(), oid), (B, r, b)
            if pers["status"][b] == O.CONVERGED:
                assert pers["relres"][b] <= 1e-6
            else:  # the iteration cap: the same residual as the multi-kernel path, to rounding
                assert pers["iters"][b] == 20
                assert abs(pers["relres"][b] - eager["relres"][b]) <= 1e-3 * eager["relres"][b]
    finally:
        c.close()


def random_graph(n, per_row, seed):
    rng = np.random.default_rng(seed)
    rows = np.repeat(np.arange(n, dtype=np.int64), per_row)
    cols = rng.integers(0, n, size=n * per_row)
    keep = rows != cols
    a = np.minimum(rows[keep], cols[keep])
    b = np.maximum(rows[keep], cols[keep])
    key = np.unique(a * n + b)
    a, b = key // n, key % n
    w = rng.uniform(0.1, 1.0, size=a.size)
    r = np.concatenate([a, b])
    c = np.concatenate([b, a])
    ww = np.concatenate([w, w])
    o = np.lexsort((c, r))
    r, c, ww = r[o], c[o], ww[o]
    rowptr = np.zeros(n + 1, np.int64)
    np.add.at(rowptr, r + 1, 1)
    return np.cumsum(rowptr), c.astype(np.int32), ww.astype(np.float32)


@pytest.mark.parametrize("B,r,mode", [(5, 37, 1), (16, 37, 1), (33, 0, 2), (64, 0, 2), (7, 0, 1)])
def test_persistent_parity_ragged(torch_dev, B, r, mode):
    """1237 items, sparse y with repeated ids, max_iter 9 and no tolerance."""
    import torch
    from paper_1807_08692_amd import hd
    N, KY = 1237, 6
    rng = np.random.default_rng(B + 100 * r)
    rowptr, col, w = random_graph(N, 5, 3)
    s32 = O.normalize(N, rowptr, col, w.astype(np.float64)).astype(np.float32)
    g = O.Graph64.from_csr(N, rowptr, col, s32)
    U = np.linalg.qr(rng.standard_normal((N, max(r, 1))))[0][:, :r].astype(np.float32)
    lam = np.sort(rng.uniform(0.0, 0.95, size=r))[::-1].copy()
    ids = rng.integers(0, N, size=(B, KY)).astype(np.int32)
    ids[0, 1] = ids[0, 0]
    vals = rng.uniform(0.1, 1.0, size=(B, KY)).astype(np.float32)
    c = hd.Context(0)
    try:
        c.load_graph(N, rowptr, col, s32)
        if r:
            c.load_eigs(U, lam, dtype="f32")
        c.set_persistent(mode)
        ti, tv = torch.from_numpy(ids).to(torch_dev), torch.from_numpy(vals).to(torch_dev)
        out = c.query_batch(None, ti, tv, alpha=0.99, max_iter=9, tol=0.0, rank_r=r, k_y=KY, top_k=10, want_x=True)
        torch.cuda.synchronize()
        assert np.all(out["iters"] == 9)
        for b in range(B):
            xo, *_ = O.iterate(g, U if r else None, lam if r else None, 0.99, ids[b], vals[b], 9, 0.0)
            x = out["x"][b].double().cpu().numpy()
            assert rel(x, xo) <= 1e-4, (b, rel(x, xo))
            oid, _ = O.rank(x, 10)
            assert np.array_equal(out["rank_ids"][b].cpu().numpy(), oid), b
        # no product: x is the spectral term alone
        z = c.query_batch(None, ti, tv, alpha=0.99, max_iter=0, tol=0.0, rank_r=r, k_y=KY, top_k=10, want_x=True)
        torch.cuda.synchronize()
        xs0 = O.iterate(g, U if r else None, lam if r else None, 0.99, ids[1], vals[1], 0, 0.0)[0]
        assert np.all(z["iters"] == 0)
        if r:
            assert rel(z["x"][1].double().cpu().numpy(), xs0) <= 1e-5
        else:
            assert np.all(z["x"][1].cpu().numpy() == 0.0)
    finally:
        c.close()


def test_persistent_plan_replays_bitwise(fx, torch_dev):
    import torch
    from paper_1807_08692_amd import hd
    c = hd.Context(0)
    try:
        c.load_graph(fx.n, fx.rowptr, fx.col, fx.s)
        c.load_eigs(fx.U, fx.lam, dtype="f32")
        c.load_descriptors(fx.V)
        c.set_persistent(1)
        kw = dict(alpha=0.99, max_iter=20, tol=1e-6, rank_r=-1, k_y=fx.cfg.k_y, top_k=30)
        plan = hd.Plan(c, 4, "descriptors", **kw)
        for rep in range(3):
            q = torch.from_numpy(fx.Q[4 * rep:4 * rep + 4]).to(torch_dev)
            ref = c.query_batch(q, **kw)
            torch.cuda.synchronize()
            got = plan.run(q)
            torch.cuda.synchronize()
            assert torch.equal(got["rank_ids"], ref["rank_ids"]) and torch.equal(got["rank_scores"], ref["rank_scores"])
            assert np.array_equal(got["iters"], ref["iters"]) and np.array_equal(got["relres"], ref["relres"])
        plan.close()
    finally:
        c.close()


def test_barrier_wait_bound_reports_and_recovers(fx, torch_dev):
    import torch
    from paper_1807_08692_amd import hd
    c = hd.Context(0)
    try:
        c.load_graph(fx.n, fx.rowptr, fx.col, fx.s)
        c.load_descriptors(fx.V)
        q = torch.from_numpy(fx.Q[:8]).to(torch_dev)
        kw = dict(alpha=0.99, max_iter=20, tol=1e-6, rank_r=0, k_y=fx.cfg.k_y, top_k=10, want_x=True)
        c.set_persistent(1, spin_limit=1)
        with pytest.raises(hd.HDError) as ei:
            c.query_batch(q, **kw)
        assert "limit" in str(ei.value)
        c.set_persistent(1)
        ok = c.query_batch(q, **kw)
        c.set_persistent(0)
        ref = c.query_batch(q, **kw)
        torch.cuda.synchronize()
        assert np.array_equal(ok["status"], ref["status"])
        for b in range(8):
            assert rel(ok["x"][b].double().cpu().numpy(), ref["x"][b].double().cpu().numpy()) <= 1e-5
    finally:
        c.close()
