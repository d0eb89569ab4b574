"""GPU tests of the first CG iteration without full fills: with the dense
bfloat16 forms of U1 and with plain CG, the query path zeroes only the
rows of R and P that y touches, and the first iteration reads R and P on
those rows alone (X nowhere) and writes all three on every row
(Section 5: CG from x0 = 0, r0 = p0 = y). A context whose solver vectors
still hold another batch's values must give bitwise the results of a fresh
context: no value of the earlier batch may reach x."""
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
    return W.build_fixture(W.CONFIGS["n5k"], n_queries=200, prefer_gpu=False)


def make_ctx(fx, form):
    from paper_1807_08692_amd import hd
    c = hd.Context(0)
    c.load_graph(fx.n, fx.rowptr, fx.col, fx.s)
    c.load_eigs(fx.U, fx.lam, dtype=form)
    c.load_descriptors(fx.V)
    return c


def run(ctx, torch_dev, Q, **kw):
    import torch
    q = torch.from_numpy(np.ascontiguousarray(Q, np.float32)).to(torch_dev)
    out = ctx.query_batch(q, want_x=True, want_y=True, **kw)
    torch.cuda.synchronize()
    return out


def run_sparse(ctx, torch_dev, ids, vals, **kw):
    import torch
    yi = torch.from_numpy(np.ascontiguousarray(ids, np.int32)).to(torch_dev)
    yv = torch.from_numpy(np.ascontiguousarray(vals, np.float32)).to(torch_dev)
    out = ctx.query_batch(None, yi, yv, want_x=True, **kw)
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("form", ["bf16x2", "fp8"])
@pytest.mark.parametrize("rank_r", [-1, 0])
@pytest.mark.parametrize("iters", [1, 2, 5])
def test_reused_workspace_matches_fresh(fx, torch_dev, form, rank_r, iters):
    kw = dict(alpha=0.99, tol=0.0, rank_r=rank_r, k_y=fx.cfg.k_y, top_k=20)
    used = make_ctx(fx, form)
    fresh = make_ctx(fx, form)
    try:
        # fill the workspace with another batch (130 columns: other row
        # stride, other rows of y), then run three queries
        run(used, torch_dev, fx.Q[:130], max_iter=7, **kw)
        a = run(used, torch_dev, fx.Q[150:153], max_iter=iters, **kw)
        b = run(fresh, torch_dev, fx.Q[150:153], max_iter=iters, **kw)
        assert np.array_equal(a["y_ids"].cpu().numpy(), b["y_ids"].cpu().numpy())
        assert np.array_equal(a["x"].cpu().numpy(), b["x"].cpu().numpy())
        assert np.array_equal(a["rank_ids"].cpu().numpy(), b["rank_ids"].cpu().numpy())
        assert np.array_equal(a["iters"], b["iters"]) and np.array_equal(a["status"], b["status"])
        # and against the oracle run on the same y
        g = O.Graph64.from_csr(fx.n, fx.rowptr, fx.col, fx.s)
        x = a["x"].cpu().numpy()
        for col in range(3):
            yi = a["y_ids"][col].cpu().numpy()
            yv = a["y_val"][col].cpu().numpy()
            if rank_r == 0:
                xo, *_ = O.iterate(g, None, None, 0.99, yi, yv, iters, 0.0)
                assert np.linalg.norm(x[col] - xo) / np.linalg.norm(xo) <= 1e-4
    finally:
        used.close()
        fresh.close()


@pytest.mark.parametrize("rank_r", [-1, 0])
def test_zero_y_after_other_batch(fx, torch_dev, rank_r):
    """A batch whose every y is zero (every column ZERO_RHS, no column
    active in the first iteration) after a batch that left values in the
    workspace: x is exactly zero beyond the spectral term, which is zero too."""
    ctx = make_ctx(fx, "bf16x2")
    try:
        kw = dict(alpha=0.99, tol=0.0, rank_r=rank_r, k_y=fx.cfg.k_y, top_k=5)
        run(ctx, torch_dev, fx.Q[:100], max_iter=6, **kw)
        rng = np.random.default_rng(4)
        ids = rng.choice(fx.n, size=(3, fx.cfg.k_y), replace=False).astype(np.int32).reshape(3, -1)
        out = run_sparse(ctx, torch_dev, ids, np.zeros(ids.shape, np.float32), max_iter=4, **kw)
        assert np.all(out["status"] == O.ZERO_RHS)
        assert not np.any(out["x"].cpu().numpy())
    finally:
        ctx.close()


def test_plan_after_other_batch(fx, torch_dev):
    """The HIP-graph form of the path (all iterations queued) after another
    batch: bitwise the eager result of a fresh context."""
    import torch
    from paper_1807_08692_amd import hd
    kw = dict(alpha=0.99, max_iter=4, tol=0.0, rank_r=-1, k_y=fx.cfg.k_y, top_k=20)
    used = make_ctx(fx, "bf16x2")
    fresh = make_ctx(fx, "bf16x2")
    try:
        run(used, torch_dev, fx.Q[:130], **dict(kw, max_iter=7))
        q = torch.from_numpy(np.ascontiguousarray(fx.Q[160:164], np.float32)).to(torch_dev)
        pl = hd.Plan(used, 4, "descriptors", **kw)
        outs = []
        for rep in range(3):
            run(used, torch_dev, fx.Q[rep * 40:rep * 40 + 70], **dict(kw, max_iter=3))
            o = pl.run(q)
            torch.cuda.synchronize()
            outs.append(o["rank_ids"].cpu().numpy().copy())
        pl.close()
        b = run(fresh, torch_dev, fx.Q[160:164], **kw)
        for r in outs:
            assert np.array_equal(r, b["rank_ids"].cpu().numpy())
    finally:
        used.close()
        fresh.close()
