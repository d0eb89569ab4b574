"""GPU tests of fixed-iteration runs without the final residual (tol < 0):
the last product updates x alone, and nothing forms the residual that no
output reads (Section 5: x_k needs p_{k-1} and the step size from
p^T A p, not r_k). x, the ranking, the iteration counts and the status
must equal those of tol = 0 bit for bit, and relres must be that of the
residual before the last product, i.e. of a run one iteration shorter."""
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
    return W.build_fixture(W.CONFIGS["n5k"], n_queries=80, prefer_gpu=False)


@pytest.fixture(scope="module", params=["bf16x2", "f32"])
def ctx(request, fx, torch_dev):
    from paper_1807_08692_amd import hd
    c = hd.Context(0)
    c.load_graph(fx.n, fx.rowptr, fx.col, fx.s)
    c.load_eigs(fx.U, fx.lam, dtype=request.param)
    c.load_descriptors(fx.V)
    yield c
    c.close()


def run(ctx, torch_dev, Q, **kw):
    import torch
    q = torch.from_numpy(np.ascontiguousarray(Q, np.float32)).to(torch_dev)
    out = ctx.query_batch(q, want_x=True, **kw)
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("rank_r", [-1, 0])
@pytest.mark.parametrize("iters", [1, 3, 6])
@pytest.mark.parametrize("B", [3, 70])
def test_no_final_residual(ctx, fx, torch_dev, rank_r, iters, B):
    kw = dict(alpha=0.99, rank_r=rank_r, k_y=fx.cfg.k_y, top_k=20)
    a = run(ctx, torch_dev, fx.Q[:B], max_iter=iters, tol=-1.0, **kw)
    b = run(ctx, torch_dev, fx.Q[:B], max_iter=iters, tol=0.0, **kw)
    assert np.array_equal(a["x"].cpu().numpy(), b["x"].cpu().numpy())
    assert np.array_equal(a["rank_ids"].cpu().numpy(), b["rank_ids"].cpu().numpy())
    assert np.array_equal(a["iters"], b["iters"]) and np.all(a["iters"] == iters)
    assert np.array_equal(a["status"], b["status"]) and np.all(a["status"] == O.MAXITER)
    if iters == 1:
        assert np.all(a["relres"] == 1.0)  # the residual before the first product is y
    else:
        c = run(ctx, torch_dev, fx.Q[:B], max_iter=iters - 1, tol=0.0, **kw)
        assert np.array_equal(a["relres"], c["relres"])


def test_plan_no_final_residual(ctx, fx, torch_dev):
    """The HIP-graph form with tol < 0 replays bitwise the eager result."""
    import torch
    from paper_1807_08692_amd import hd
    kw = dict(alpha=0.99, max_iter=4, tol=-1.0, rank_r=-1, k_y=fx.cfg.k_y, top_k=20)
    e = run(ctx, torch_dev, fx.Q[:5], **kw)
    q = torch.from_numpy(np.ascontiguousarray(fx.Q[:5], np.float32)).to(torch_dev)
    pl = hd.Plan(ctx, 5, "descriptors", **kw)
    try:
        for rep in range(3):
            o = pl.run(q)
            torch.cuda.synchronize()
            assert np.array_equal(o["rank_ids"].cpu().numpy(), e["rank_ids"].cpu().numpy())
            assert np.array_equal(o["relres"], e["relres"]) and np.array_equal(o["iters"], e["iters"])
    finally:
        pl.close()
