"""GPU tests of query plans (the whole query path captured into a HIP graph
and replayed): every replay equals hd_query_batch on the same input bit for
bit (rankings, scores, iteration counts, statuses, residuals), with eager
queries on other inputs between the replays, after the context's workspace
has moved (the plan captures itself again), and with y given directly."""
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
    return W.build_fixture(W.CONFIGS["n5k"], n_queries=400, prefer_gpu=False)


@pytest.fixture(scope="module", params=["f32", "bf16x2", "bf16"])
def ctx(request, fx, torch_dev):
    from paper_1807_08692_amd import hd
    c = hd.Context(0)
    c.load_graph(fx.n, fx.rowptr, fx.col, fx.s)
    c.load_eigs(fx.U, fx.lam, dtype=request.param)
    c.load_descriptors(fx.V, dtype="f32")
    yield c
    c.close()


def same(pr, eg):
    assert np.array_equal(pr["iters"], eg["iters"])
    assert np.array_equal(pr["status"], eg["status"])
    assert np.array_equal(pr["relres"], eg["relres"])
    assert np.array_equal(pr["rank_ids"].cpu().numpy(), eg["rank_ids"].cpu().numpy())
    assert np.array_equal(pr["rank_scores"].cpu().numpy(), eg["rank_scores"].cpu().numpy())


@pytest.mark.parametrize("B,max_iter,tol", [(5, 20, 1e-6), (130, 20, 1e-6), (64, 4, 0.0)])
def test_plan_replays_match_eager(ctx, fx, torch_dev, B, max_iter, tol):
    import torch
    from paper_1807_08692_amd import hd
    kw = dict(alpha=0.99, max_iter=max_iter, tol=tol, rank_r=-1, k_y=fx.cfg.k_y, top_k=50)
    plan = hd.Plan(ctx, B, "descriptors", **kw)
    try:
        for rep in range(4):
            q = torch.from_numpy(fx.Q[rep * 50: rep * 50 + B]).to(torch_dev)
            pr = plan.run(q)
            torch.cuda.synchronize()
            eg = ctx.query_batch(q, **kw)
            torch.cuda.synchronize()
            same(pr, eg)
            # eager work on another input between replays
            other = torch.from_numpy(fx.Q[300:307]).to(torch_dev)
            ctx.query_batch(other, **kw)
            torch.cuda.synchronize()
    finally:
        plan.close()


def test_plan_recaptures_after_workspace_moves(ctx, fx, torch_dev):
    import torch
    from paper_1807_08692_amd import hd
    kw = dict(alpha=0.99, max_iter=20, tol=1e-6, rank_r=-1, k_y=fx.cfg.k_y, top_k=20)
    plan = hd.Plan(ctx, 40, "descriptors", **kw)
    try:
        q = torch.from_numpy(fx.Q[:40]).to(torch_dev)
        first = plan.run(q)
        ids0 = first["rank_ids"].cpu().numpy().copy()
        # a wider batch grows (moves) the context's workspace
        big = torch.from_numpy(fx.Q[:400]).to(torch_dev)
        ctx.query_batch(big, **kw)
        torch.cuda.synchronize()
        again = plan.run(q)
        assert np.array_equal(again["rank_ids"].cpu().numpy(), ids0)
        same(again, ctx.query_batch(q, **kw))
        # a changed launch parameter is picked up too
        ctx.set_tuning("spmm_cpl", 1)
        third = plan.run(q)
        ctx.set_tuning("spmm_cpl", 0)
        assert np.array_equal(third["rank_ids"].cpu().numpy(), ids0)
    finally:
        plan.close()


def test_plan_with_y_input(ctx, fx, torch_dev):
    import torch
    from paper_1807_08692_amd import hd
    B = 9
    ids, vals = [], []
    for q in fx.Q[:B]:
        i, v = O.observation(fx.V, q, fx.cfg.k_y)
        ids.append(i)
        vals.append(v)
    yi = torch.from_numpy(np.stack(ids).astype(np.int32)).to(torch_dev)
    yv = torch.from_numpy(np.stack(vals).astype(np.float32)).to(torch_dev)
    kw = dict(alpha=0.99, max_iter=20, tol=1e-6, rank_r=-1, k_y=fx.cfg.k_y, top_k=30)
    plan = hd.Plan(ctx, B, "y", **kw)
    try:
        for _ in range(2):
            pr = plan.run(y_ids=yi, y_val=yv)
            same(pr, ctx.query_batch(None, yi, yv, **kw))
        bad = yi.clone()
        bad[3, 0] = fx.n
        with pytest.raises(hd.HDError):
            plan.run(y_ids=bad, y_val=yv)
    finally:
        plan.close()
