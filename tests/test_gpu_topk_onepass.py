"""GPU tests of the one-pass top-K (HD_TUNE_TOPK_ONEPASS): the top-k_y of
the similarities and the final top-K taken from candidates emitted by the
kernels that produce the scores, with a sampled threshold per row, against
the two-pass form (score matrix, then selection) on the same inputs. Both
forms select exactly, so every output must agree bit for bit: y ids and
values, iteration counts, ranking ids and scores. Rows whose candidate
lists cannot give the top-K go to the exact fallback; the tie tests force
that path (all scores equal, or many items with the query's own
descriptor) and check the ties go to the lowest ids."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

N = 70_001          # above the one-pass minimum, not a multiple of 16, 64 or 256
D = 96
R = 64
KY = 10
TOPK = 100


def random_graph(n, per_row, seed):
    rng = np.random.default_rng(seed)
    rows = np.repeat(np.arange(n, dtype=np.int64), per_row)
    cols = rng.integers(0, n, size=n * per_row)
    keep = rows != cols
    rows, cols = rows[keep], cols[keep]
    a = np.minimum(rows, cols)
    b = np.maximum(rows, cols)
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


def unit_rows(a):
    return (a / np.linalg.norm(a, axis=1, keepdims=True)).astype(np.float32)


@pytest.fixture(scope="module")
def data():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rng = np.random.default_rng(1807)
    rowptr, col, w = random_graph(N, 5, 11)
    V = unit_rows(rng.standard_normal((N, D)))
    Q = unit_rows(rng.standard_normal((256, D)))
    U = (rng.standard_normal((N, R)) / np.sqrt(N)).astype(np.float32)
    lam = np.sort(rng.uniform(0.0, 0.9, R))[::-1].copy()
    return rowptr, col, w, V, Q, U, lam


def make_ctx(data, u_dtype, v_dtype, V=None):
    from paper_1807_08692_amd import hd
    rowptr, col, w, V0, Q, U, lam = data
    c = hd.Context(0)
    c.load_graph(N, rowptr, col, w, normalize=True)
    c.load_eigs(U, lam, dtype=u_dtype)
    c.load_descriptors(V0 if V is None else V, dtype=v_dtype)
    return c


def run(ctx, onepass, q=None, y_ids=None, y_val=None, rank_r=-1, max_iter=5):
    import torch
    ctx.set_tuning("topk_onepass", onepass)
    out = ctx.query_batch(q, y_ids, y_val, alpha=0.99, max_iter=max_iter, tol=0.0, rank_r=rank_r, k_y=KY,
                          top_k=TOPK, want_y=q is not None)
    torch.cuda.synchronize()
    res = {k: (v.cpu().numpy() if hasattr(v, "cpu") else np.array(v)) for k, v in out.items()}
    ctx.set_tuning("topk_onepass", 0)
    return res


def assert_same(a, b, what):
    for k in a:
        assert np.array_equal(a[k], b[k]), (what, k)


@pytest.mark.parametrize("u_dtype,v_dtype", [("bf16x2", "bf16"), ("bf16", "fp8"), ("fp8", "bf16")])
@pytest.mark.parametrize("B", [100, 256])
def test_onepass_equals_twopass(data, u_dtype, v_dtype, B):
    import torch
    dev = torch.device("cuda:0")
    q = torch.from_numpy(data[4][:B]).to(dev)
    with make_ctx(data, u_dtype, v_dtype) as ctx:
        for rank_r in (-1, 0):
            ctx.timing_enable(True)
            one = run(ctx, 2, q, rank_r=rank_r)
            t1 = ctx.timing()
            ctx.timing_enable(False)
            two = run(ctx, 1, q, rank_r=rank_r)
            assert_same(one, two, (u_dtype, v_dtype, B, rank_r))
            # the one-pass form ran: sample + thresholds + lists + gated
            # fallback launches around the one similarity launch
            assert t1["sim"][1] == 1 and t1["topk_y"][1] == 5, t1
            assert t1["topk_rank"][1] >= 4, t1
            # the default setting is the one-pass form
            assert_same(run(ctx, 0, q, rank_r=rank_r), one, ("default", rank_r))


def test_onepass_in_plan_replays(data):
    import torch
    from paper_1807_08692_amd import hd
    dev = torch.device("cuda:0")
    B = 64
    q = torch.from_numpy(data[4][:B]).to(dev)
    with make_ctx(data, "bf16x2", "bf16") as ctx:
        ref = run(ctx, 2, q)
        p = hd.Plan(ctx, B, "descriptors", alpha=0.99, max_iter=5, tol=0.0, rank_r=-1, k_y=KY, top_k=TOPK)
        try:
            for _ in range(3):
                out = p.run(q)
                torch.cuda.synchronize()
                assert np.array_equal(out["rank_ids"].cpu().numpy(), ref["rank_ids"])
                assert np.array_equal(out["rank_scores"].cpu().numpy(), ref["rank_scores"])
                # eager work between replays
                run(ctx, 1, q[:8])
        finally:
            p.close()


@pytest.mark.parametrize("u_dtype,rank_r", [("bf16x2", -1), ("bf16", 0)])
def test_rank_fallback_all_ties(data, u_dtype, rank_r):
    """y = 0: every x is 0, every item passes the threshold, the lists
    overflow and each row is selected exactly: ids 0..K-1, scores 0."""
    import torch
    dev = torch.device("cuda:0")
    B = 70
    rng = np.random.default_rng(3)
    ids = torch.from_numpy(np.stack([rng.choice(N, KY, replace=False) for _ in range(B)]).astype(np.int32)).to(dev)
    vals = torch.zeros((B, KY), dtype=torch.float32, device=dev)
    with make_ctx(data, u_dtype, "bf16") as ctx:
        one = run(ctx, 2, None, ids, vals, rank_r=rank_r)
        two = run(ctx, 1, None, ids, vals, rank_r=rank_r)
        assert_same(one, two, ("ties", u_dtype, rank_r))
        assert np.array_equal(one["rank_ids"], np.tile(np.arange(TOPK, dtype=np.int32), (B, 1)))
        assert not one["rank_scores"].any()


def test_y_fallback_duplicated_descriptors(data):
    """20,000 items carry query 0's own descriptor: row 0's similarities tie
    at the top beyond the candidate capacity (fallback, ties to the lowest
    ids); the other rows take the lists."""
    import torch
    dev = torch.device("cuda:0")
    V = data[3].copy()
    Q = data[4][:40].copy()
    dup = np.arange(5, 5 + 20_000) * 3 + 1
    V[dup] = Q[0]
    q = torch.from_numpy(Q).to(dev)
    with make_ctx(data, "bf16x2", "bf16", V=V) as ctx:
        one = run(ctx, 2, q)
        two = run(ctx, 1, q)
        assert_same(one, two, "dup")
        assert np.array_equal(one["y_ids"][0], dup[:KY].astype(np.int32))
        assert np.all(one["y_val"][0] == one["y_val"][0][0])
