"""GPU tests of the continuous-batching server: a request gives the same
result alone and in a busy server (joining while other columns are mid-way
through their solves), matches the batch path and the oracle, honours its own
iteration cap, and the HBM budget sets the column count."""
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
def ctx(fx, torch_dev):
    from paper_1807_08692_amd import hd
    c = hd.Context(0)
    c.load_graph(fx.n, fx.rowptr, fx.col, fx.s)
    c.load_eigs(fx.U, fx.lam)
    c.load_descriptors(fx.V)
    yield c
    c.close()


def ys(fx, idx):
    ids, vals = [], []
    for q in fx.Q[idx]:
        i, v = O.observation(fx.V, q, fx.cfg.k_y)
        ids.append(i)
        vals.append(v)
    return np.stack(ids).astype(np.int32), np.stack(vals).astype(np.float32)


def drain(srv, want, results, max_steps=200):
    for _ in range(max_steps):
        if len(results) >= want:
            return
        srv.step(1)
        res = srv.poll()
        for k, t in enumerate(res["tickets"]):
            results[int(t)] = {key: res[key][k] for key in ("ids", "scores", "iters", "relres", "status")}
    raise AssertionError("server did not finish")


def test_alone_equals_in_mix(fx, ctx):
    from paper_1807_08692_amd import hd
    ids, vals = ys(fx, np.arange(30))
    kw = dict(alpha=0.99, max_iter=20, tol=1e-6, rank_r=50, k_y=fx.cfg.k_y, top_k=50)
    with_alone = {}
    srv = hd.Server(ctx, 32, **kw)
    t = srv.submit(ids[7:8], vals[7:8])
    drain(srv, 1, with_alone)
    alone = with_alone[int(t[0])]
    srv.close()
    # busy server: 12 requests start, two steps later 18 more join (incl. #7)
    srv = hd.Server(ctx, 32, **kw)
    res = {}
    t_first = srv.submit(ids[:7], vals[:7])
    srv.submit(ids[8:13], vals[8:13])
    srv.step(2)
    t_join = srv.submit(ids[7:8], vals[7:8])
    srv.submit(ids[13:30], vals[13:30])
    assert srv.in_use == 30
    drain(srv, 30, res)
    mixed = res[int(t_join[0])]
    assert np.array_equal(mixed["ids"], alone["ids"])
    assert np.array_equal(mixed["scores"], alone["scores"])
    assert mixed["iters"] == alone["iters"]
    assert srv.in_use == 0
    srv.close()


def test_server_matches_batch_and_oracle(fx, ctx, torch_dev):
    import torch
    from paper_1807_08692_amd import hd
    ids, vals = ys(fx, np.arange(5))
    kw = dict(alpha=0.99, max_iter=20, tol=1e-6, rank_r=50, k_y=fx.cfg.k_y, top_k=50)
    srv = hd.Server(ctx, 8, **kw)
    tk = srv.submit(ids, vals)
    res = {}
    drain(srv, 5, res)
    srv.close()
    out = ctx.query_batch(None, torch.from_numpy(ids).to(torch_dev), torch.from_numpy(vals).to(torch_dev),
                          want_x=True, **kw)
    torch.cuda.synchronize()
    g = O.Graph64.from_csr(fx.n, fx.rowptr, fx.col, fx.s)
    for b in range(5):
        r = res[int(tk[b])]
        assert r["iters"] == out["iters"][b] and r["status"] == O.CONVERGED
        xo, *_ = O.iterate(g, fx.U, fx.lam, 0.99, ids[b], vals[b], int(r["iters"]), 0.0)
        # scores of the ranked items agree with the oracle's x
        assert np.allclose(r["scores"], xo[r["ids"]], rtol=2e-4, atol=1e-9 * np.abs(xo).max())
        # and with the batch path (same rounding up to the first product's coefficients)
        assert np.allclose(r["scores"], out["rank_scores"].cpu().numpy()[b], rtol=1e-5, atol=1e-12)


@pytest.mark.parametrize("dtype", ["bf16", "bf16x2", "fp8"])
def test_server_bf16_forms_match_batch(fx, torch_dev, dtype):
    """The server with bfloat16 (one- and two-term) U1: same ranking as the
    batch path with the same storage, scores within fp32 rounding."""
    import torch
    from paper_1807_08692_amd import hd
    c = hd.Context(0)
    try:
        c.load_graph(fx.n, fx.rowptr, fx.col, fx.s)
        c.load_eigs(fx.U, fx.lam, dtype=dtype)
        ids, vals = ys(fx, np.arange(6))
        kw = dict(alpha=0.99, max_iter=20, tol=1e-6, rank_r=50, k_y=fx.cfg.k_y, top_k=50)
        srv = hd.Server(c, 8, **kw)
        tk = srv.submit(ids, vals)
        res = {}
        drain(srv, 6, res)
        srv.close()
        out = c.query_batch(None, torch.from_numpy(ids).to(torch_dev),
                            torch.from_numpy(vals).to(torch_dev), **kw)
        torch.cuda.synchronize()
        for b in range(6):
            r = res[int(tk[b])]
            assert r["iters"] == out["iters"][b]
            assert np.allclose(r["scores"], out["rank_scores"].cpu().numpy()[b], rtol=1e-5, atol=1e-12)
    finally:
        c.close()


def test_per_request_cap_and_descriptors(fx, ctx):
    from paper_1807_08692_amd import hd
    srv = hd.Server(ctx, 16, alpha=0.99, max_iter=20, tol=1e-6, rank_r=-1, k_y=fx.cfg.k_y, top_k=20)
    tk = srv.submit(q_desc=fx.Q[:6], max_iter=[2, 0, 20, 5, 20, 1])
    res = {}
    drain(srv, 6, res)
    got = [res[int(t)] for t in tk]
    assert [r["iters"] for r in got[:2]] == [2, 0]
    assert got[0]["status"] == O.MAXITER and got[1]["status"] == O.MAXITER
    assert got[2]["status"] == O.CONVERGED
    assert got[3]["iters"] == 5 and got[5]["iters"] == 1
    srv.close()


def test_hbm_budget_sets_columns(fx, ctx):
    from paper_1807_08692_amd import hd
    with pytest.raises(hd.HDError):
        hd.Server(ctx, 64, hbm_budget_bytes=1 << 20, k_y=fx.cfg.k_y, top_k=10)
    big = hd.Server(ctx, 512, k_y=fx.cfg.k_y, top_k=10)
    assert big.slots == 512
    big.close()
    col = hd.Server.column_bytes(ctx, k_y=fx.cfg.k_y, top_k=10)
    assert col > 20 * fx.n  # at least the five solver vectors
    for budget_cols, want in ((100, 64), (300, 256), (5000, 512)):
        s = hd.Server(ctx, 512, hbm_budget_bytes=budget_cols * col, k_y=fx.cfg.k_y, top_k=10)
        assert s.slots == want
        s.close()
    with pytest.raises(hd.HDError):
        hd.Server(ctx, 512, hbm_budget_bytes=63 * col, k_y=fx.cfg.k_y, top_k=10)


def test_request_loop_poisson(fx, ctx):
    """The serving loop over two servers (plain CG and hybrid on the same
    graph): every request finishes, with latencies measured."""
    from paper_1807_08692_amd import hd, serve
    ids, vals = ys(fx, np.arange(40))
    arr = serve.poisson_arrivals(2000.0, 40, seed=3)
    reqs = [serve.Request(i, float(arr[i]), "plain" if i % 2 else "hybrid", ids[i], vals[i], max_iter=100)
            for i in range(40)]
    servers = {"plain": hd.Server(ctx, 16, rank_r=0, k_y=fx.cfg.k_y, top_k=10, tol=1e-6),
               "hybrid": hd.Server(ctx, 16, rank_r=50, k_y=fx.cfg.k_y, top_k=10, tol=1e-6)}
    reqs, wall = serve.run(servers, reqs)
    st = serve.latency_stats(reqs)
    assert st["count"] == 40 and all(r.finished >= r.arrival for r in reqs)
    assert all(r.result["status"] == O.CONVERGED for r in reqs)
    for s in servers.values():
        s.close()


def _small_db(n, r, d, seed):
    """A resident database for the multi-database test: a random symmetric
    graph (about 10 entries per row), unit descriptors with normal entries and
    an orthonormal U1 with disjoint column supports, eigenvalues in [0, 0.95)."""
    rng = np.random.default_rng(seed)
    rows = np.repeat(np.arange(n, dtype=np.int64), 5)
    cols = rng.integers(0, n, size=rows.size)
    keep = rows != cols
    a, b = np.minimum(rows[keep], cols[keep]), np.maximum(rows[keep], cols[keep])
    key = np.unique(a * n + b)
    a, b = key // n, key % n
    w = rng.uniform(0.1, 1.0, size=a.size)
    rr, cc, ww = np.concatenate([a, b]), np.concatenate([b, a]), np.concatenate([w, w])
    o = np.lexsort((cc, rr))
    rr, cc, ww = rr[o], cc[o], ww[o]
    rowptr = np.zeros(n + 1, np.int64)
    np.add.at(rowptr, rr + 1, 1)
    rowptr = np.cumsum(rowptr)
    comp = rng.permutation(n) % r
    vals = rng.standard_normal(n)
    norms = np.zeros(r)
    np.add.at(norms, comp, vals ** 2)
    vals /= np.sqrt(norms[comp])
    U = np.zeros((n, r), np.float32)
    U[np.arange(n), comp] = vals
    lam = np.sort(rng.uniform(0.0, 0.95, size=r))[::-1].copy()
    V = rng.standard_normal((n, d)).astype(np.float32)
    V /= np.linalg.norm(V, axis=1, keepdims=True)
    return rowptr, cc.astype(np.int32), ww.astype(np.float32), U, lam, V


def test_three_databases_poisson(torch_dev):
    """The serving configuration at test scale: three resident databases of
    different sizes and ranks on one device, seeded Poisson arrivals routed
    uniformly to them, per-request iteration caps drawn from 5..20. Every
    request finishes with its own cap and the ranking the batch path gives for
    the same query and cap."""
    import torch
    from paper_1807_08692_amd import hd, serve
    d, ky, K = 64, 10, 10
    dbs = {"small": (2000, 16), "medium": (4000, 32), "large": (8000, 64)}
    ctxs, servers, qs = {}, {}, {}
    try:
        for t, (name, (n, r)) in enumerate(dbs.items()):
            rowptr, col, w, U, lam, V = _small_db(n, r, d, 100 + t)
            c = hd.Context(0)
            ctxs[name] = c
            c.load_graph(n, rowptr, col, w, normalize=True)
            c.load_eigs(U, lam, dtype="bf16x2")
            c.load_descriptors(V)
            servers[name] = hd.Server(c, 32, max_iter=20, tol=0.0, k_y=ky, top_k=K)
            qs[name] = np.random.default_rng(200 + t).standard_normal((40, d)).astype(np.float32)
        rng = np.random.default_rng(5)
        names = list(dbs)
        m = 90
        arr = serve.poisson_arrivals(2000.0, m, seed=9)
        route = rng.integers(0, 3, size=m)
        caps = rng.integers(5, 21, size=m)
        reqs = [serve.Request(i, float(arr[i]), names[route[i]], q_desc=qs[names[route[i]]][i % 40],
                              max_iter=int(caps[i])) for i in range(m)]
        reqs, wall = serve.run(servers, reqs)
        st = serve.latency_stats(reqs)
        assert st["count"] == m and all(r.finished >= r.arrival for r in reqs)
        for rq in reqs:
            res = rq.result
            assert res["iters"] == rq.max_iter and res["status"] == O.MAXITER
            q = torch.from_numpy(qs[rq.db][rq.rid % 40][None, :]).to(torch_dev)
            out = ctxs[rq.db].query_batch(q, alpha=0.99, max_iter=rq.max_iter, tol=0.0, k_y=ky, top_k=K)
            torch.cuda.synchronize()
            assert np.array_equal(res["ids"], out["rank_ids"][0].cpu().numpy()), (rq.db, rq.rid)
            assert np.allclose(res["scores"], out["rank_scores"][0].cpu().numpy(), rtol=1e-5, atol=1e-12)
    finally:
        for s in servers.values():
            s.close()
        for c in ctxs.values():
            c.close()


def test_cancel_leaves_other_columns_bitwise(fx, ctx):
    """Requests cancelled in the middle of their solves never come back, free
    their columns at once, and every other request's result is bit for bit
    what it is in the same run without the cancellations; a request admitted
    into a freed column gets its result alone."""
    from paper_1807_08692_amd import hd
    ids, vals = ys(fx, np.arange(31))
    kw = dict(alpha=0.99, max_iter=20, tol=1e-6, rank_r=50, k_y=fx.cfg.k_y, top_k=50)

    def run(cancel):
        srv = hd.Server(ctx, 32, **kw)
        res = {}
        tk = srv.submit(ids[:30], vals[:30])
        srv.step(2)
        late = None
        if cancel:
            gone = [int(tk[q]) for q in (3, 4, 17, 29)]
            assert srv.cancel(gone + [10 ** 9]) == 4  # an unknown ticket is ignored
            assert srv.in_use == 26
            assert srv.cancel(gone) == 0
            late = srv.submit(ids[30:31], vals[30:31])
            assert srv.in_use == 27
        drain(srv, 27 if cancel else 30, res)
        assert srv.in_use == 0
        srv.close()
        return tk, res, late

    tk0, full, _ = run(False)
    tk1, part, late = run(True)
    cancelled = {int(tk1[q]) for q in (3, 4, 17, 29)}
    assert not cancelled & set(part)
    for q in range(30):
        if int(tk1[q]) in cancelled:
            continue
        a, b = full[int(tk0[q])], part[int(tk1[q])]
        assert np.array_equal(a["ids"], b["ids"]) and np.array_equal(a["scores"], b["scores"]), q
        assert a["iters"] == b["iters"] and a["relres"] == b["relres"], q
    alone = {}
    srv = hd.Server(ctx, 32, **kw)
    t = srv.submit(ids[30:31], vals[30:31])
    drain(srv, 1, alone)
    srv.close()
    assert np.array_equal(alone[int(t[0])]["scores"], part[int(late[0])]["scores"])


def test_repeated_y_ids_alone_equals_mix(fx, ctx):
    """A y whose ids repeat (three and four times: their values add) gives
    bit for bit the same result alone and in a busy server, and the oracle's
    result for the summed y."""
    from paper_1807_08692_amd import hd
    ids, vals = ys(fx, np.arange(20))
    ids[5, 1:4] = ids[5, 0]          # one id four times
    ids[5, 6:9] = ids[5, 5]          # another three times
    kw = dict(alpha=0.99, max_iter=20, tol=1e-6, rank_r=50, k_y=fx.cfg.k_y, top_k=50)
    alone = {}
    srv = hd.Server(ctx, 32, **kw)
    t = srv.submit(ids[5:6], vals[5:6])
    drain(srv, 1, alone)
    srv.close()
    a = alone[int(t[0])]
    for rep in range(2):
        srv = hd.Server(ctx, 32, **kw)
        res = {}
        tk = srv.submit(ids[:5], vals[:5])
        srv.step(1 + rep)
        tj = srv.submit(ids[5:20], vals[5:20])
        drain(srv, 20, res)
        srv.close()
        m = res[int(tj[0])]
        assert np.array_equal(m["ids"], a["ids"]) and np.array_equal(m["scores"], a["scores"])
        assert m["iters"] == a["iters"]
    g = O.Graph64.from_csr(fx.n, fx.rowptr, fx.col, fx.s)
    xo, *_ = O.iterate(g, fx.U, fx.lam, 0.99, ids[5], vals[5], int(a["iters"]), 0.0)
    assert np.allclose(a["scores"], xo[a["ids"]], rtol=2e-4, atol=1e-9 * np.abs(xo).max())


def test_bad_y_id_admits_nothing(fx, ctx):
    """A submission with an id outside [0, n) is rejected before any column
    changes: nothing is admitted and the server keeps working."""
    from paper_1807_08692_amd import hd
    ids, vals = ys(fx, np.arange(4))
    kw = dict(alpha=0.99, max_iter=20, tol=1e-6, rank_r=50, k_y=fx.cfg.k_y, top_k=50)
    srv = hd.Server(ctx, 8, **kw)
    bad = ids.copy()
    bad[2, 3] = fx.n
    with pytest.raises(hd.HDError):
        srv.submit(bad, vals)
    assert srv.in_use == 0
    tk = srv.submit(ids, vals)
    res = {}
    drain(srv, 4, res)
    assert set(res) == {int(t) for t in tk}
    srv.close()


@pytest.fixture(scope="module")
def ctx_bf16x2(fx, torch_dev):
    from paper_1807_08692_amd import hd
    c = hd.Context(0)
    c.load_graph(fx.n, fx.rowptr, fx.col, fx.s)
    c.load_eigs(fx.U, fx.lam, dtype="bf16x2")
    yield c
    c.close()


def alone_results(ctx, ids, vals, caps, kw):
    from paper_1807_08692_amd import hd
    out = []
    for q in range(len(ids)):
        srv = hd.Server(ctx, 8, **kw)
        t = srv.submit(ids[q:q + 1], vals[q:q + 1], max_iter=[int(caps[q])])
        res = {}
        drain(srv, 1, res)
        srv.close()
        out.append(res[int(t[0])])
    return out


def same(a, b):
    return (np.array_equal(a["ids"], b["ids"]) and np.array_equal(a["scores"], b["scores"])
            and a["iters"] == b["iters"] and a["relres"] == b["relres"] and a["status"] == b["status"])


def test_bf16_column_reuse_alone_equals_mix(fx, ctx_bf16x2):
    """Two-term bf16 U1 (the server whose x/p update clears the columns of
    finished requests): 24 requests with caps 2..9 through 8 columns, so
    every column is reused several times, each admitted right after a poll
    freed it; one request has y = 0 (zero right-hand side, stopped at
    admission). Every result equals the request's result alone, bit for bit."""
    from paper_1807_08692_amd import hd
    ids, vals = ys(fx, np.arange(24))
    vals[5] = 0.0
    caps = 2 + (np.arange(24) * 7) % 8
    kw = dict(alpha=0.99, max_iter=20, tol=1e-6, rank_r=50, k_y=fx.cfg.k_y, top_k=50)
    ref = alone_results(ctx_bf16x2, ids, vals, caps, kw)
    srv = hd.Server(ctx_bf16x2, 8, **kw)
    res, tick, nxt = {}, {}, 0
    for _ in range(400):
        if nxt < 24 and srv.in_use < 8:
            k = min(8 - srv.in_use, 24 - nxt, 3)
            tk = srv.submit(ids[nxt:nxt + k], vals[nxt:nxt + k], max_iter=[int(c) for c in caps[nxt:nxt + k]])
            for j, t in enumerate(tk):
                tick[int(t)] = nxt + j
            nxt += len(tk)
        srv.step(1)
        r = srv.poll()
        for k, t in enumerate(r["tickets"]):
            res[int(t)] = {key: r[key][k] for key in ("ids", "scores", "iters", "relres", "status")}
        if len(res) == 24:
            break
    srv.close()
    assert len(res) == 24
    for t, q in tick.items():
        assert same(res[t], ref[q]), q
    assert res[[t for t, q in tick.items() if q == 5][0]]["status"] == 2  # zero right-hand side


def test_bf16_cancel_then_readmit(fx, ctx_bf16x2):
    """A request admitted into the column of one cancelled a moment before
    (no step in between: the column still holds the cancelled request's
    vectors) gets its result alone, bit for bit, and so do the others."""
    from paper_1807_08692_amd import hd
    ids, vals = ys(fx, np.arange(12))
    caps = [20] * 12
    kw = dict(alpha=0.99, max_iter=20, tol=1e-6, rank_r=50, k_y=fx.cfg.k_y, top_k=50)
    ref = alone_results(ctx_bf16x2, ids, vals, caps, kw)
    srv = hd.Server(ctx_bf16x2, 9, **kw)
    assert srv.slots == 9
    tk = srv.submit(ids[:8], vals[:8])
    srv.step(3)
    assert srv.cancel([int(tk[2]), int(tk[5])]) == 2
    late = srv.submit(ids[8:10], vals[8:10])  # into the two cancelled columns
    assert len(late) == 2
    srv.step(2)
    assert srv.cancel([int(tk[0])]) == 1
    late2 = srv.submit(ids[10:12], vals[10:12])  # one into the cancelled column, one into the unused ninth
    assert len(late2) == 2
    res = {}
    drain(srv, 9, res)
    srv.close()
    for q, t in [(1, tk[1]), (3, tk[3]), (4, tk[4]), (6, tk[6]), (7, tk[7]),
                 (8, late[0]), (9, late[1]), (10, late2[0]), (11, late2[1])]:
        assert same(res[int(t)], ref[q]), q
