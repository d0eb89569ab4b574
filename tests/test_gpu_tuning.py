"""GPU tests of the launch parameters and the autotuner: every setting of
the search space gives the same results (the parameters only change which
lanes and waves own which columns, not the order of any sum), and the
autotuner keeps one of the valid values."""
import numpy as np
import pytest

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
    return W.build_fixture(W.CONFIGS["n5k"], n_queries=300, prefer_gpu=False)


@pytest.fixture(scope="module", params=["bf16x2", "bf16", "f32"])
def ctx(request, fx, torch_dev):
    from paper_1807_08692_amd import hd
    c = hd.Context(0)
    c.load_graph(fx.n, fx.rowptr, fx.col, fx.s)
    c.load_eigs(fx.U, fx.lam, dtype=request.param)
    c.load_descriptors(fx.V, dtype="f32")
    yield c
    c.close()


def run(ctx, fx, torch_dev, B):
    import torch
    q = torch.from_numpy(fx.Q[:B]).to(torch_dev)
    out = ctx.query_batch(q, alpha=0.99, max_iter=12, tol=1e-6, rank_r=-1, k_y=fx.cfg.k_y,
                          top_k=50, want_x=True)
    torch.cuda.synchronize()
    return out["x"].cpu().numpy(), out["rank_ids"].cpu().numpy(), out["iters"].copy()


KEYS = ("spmm_cpl", "utp_nt", "uc_nt", "spmm_bands", "topk_onepass")
VALUES = {"spmm_cpl": (1, 2, 4), "utp_nt": (1, 2, 4), "uc_nt": (1, 2, 4), "spmm_bands": (1, 2, 4, 8),
          "topk_onepass": (1, 2)}


@pytest.mark.parametrize("B", [40, 130, 300])
def test_every_setting_same_result(ctx, fx, torch_dev, B):
    for k in KEYS:
        ctx.set_tuning(k, 0)
    x0, r0, it0 = run(ctx, fx, torch_dev, B)
    for key in KEYS:
        for v in VALUES[key]:
            ctx.set_tuning(key, v)
            x, r, it = run(ctx, fx, torch_dev, B)
            ctx.set_tuning(key, 0)
            assert np.array_equal(it, it0), (key, v)
            assert np.array_equal(r, r0), (key, v)
            assert np.array_equal(x, x0), (key, v, float(np.abs(x - x0).max()))
    # source bands together with every column tiling of the sparse product
    for cpl in (1, 2, 4):
        for bands in (2, 8):
            ctx.set_tuning("spmm_cpl", cpl)
            ctx.set_tuning("spmm_bands", bands)
            x, r, it = run(ctx, fx, torch_dev, B)
            ctx.set_tuning("spmm_cpl", 0)
            ctx.set_tuning("spmm_bands", 0)
            assert np.array_equal(x, x0) and np.array_equal(r, r0) and np.array_equal(it, it0), (cpl, bands)


def test_autotune_keeps_valid_values(ctx, fx, torch_dev):
    for k in KEYS:
        ctx.set_tuning(k, 0)
    x0, r0, _ = run(ctx, fx, torch_dev, 200)
    res = ctx.autotune(256, reps=2)
    for key, rec in res.items():
        assert rec["chosen"] in (0,) + VALUES[key]
        for v, ms in rec["times_ms"].items():
            assert ms > 0.0
    assert res["spmm_cpl"]["chosen"] in (1, 2, 4)
    assert res["spmm_bands"]["chosen"] in (1, 2, 4, 8)
    assert len(res["spmm_bands"]["times_ms"]) == 4
    assert res["topk_onepass"]["times_ms"] == {} and res["topk_onepass"]["chosen"] == 0
    x, r, _ = run(ctx, fx, torch_dev, 200)
    assert np.array_equal(r, r0) and np.array_equal(x, x0)


def test_set_tuning_rejects_bad_values(ctx):
    from paper_1807_08692_amd import hd
    with pytest.raises(hd.HDError):
        ctx.set_tuning("spmm_cpl", 3)
    with pytest.raises(hd.HDError):
        ctx.set_tuning("spmm_cpl", 8)
    with pytest.raises(hd.HDError):
        ctx.set_tuning("spmm_bands", 3)
    with pytest.raises(hd.HDError):
        ctx.set_tuning("spmm_bands", 16)
    with pytest.raises(hd.HDError):
        ctx.set_tuning("topk_onepass", 3)
    with pytest.raises(hd.HDError):
        ctx.set_tuning("topk_onepass", 4)
    assert ctx.get_tuning("spmm_cpl") in (0, 1, 2, 4)
    assert ctx.get_tuning("spmm_bands") in (0, 1, 2, 4, 8)
