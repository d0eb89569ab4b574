"""GPU parity of the FP8 storage form (OCP FP8 E4M3 codes with one fp32
scale per eigenvector column or per descriptor row, converted to bfloat16 in
registers; fp32 accumulation, double CG scalars).

The oracle is given the dequantized U1 (scale times code value, in double),
so the GPU must match it to the fp32 bar (relative L2 error <= 1e-4): the
code values are exact in bfloat16 and the fp32 operands are split hi + lo.
The neighbour sets are checked against FP64 cosines of the dequantized
descriptors. The paper computes in double, so the form's effect on accuracy
is not pinned by it; it is reported against the fp32 U1 with a loose bound
that only catches a wrong scale or code order.

Cases: every stored operand padded (1237 items, r = 37, d = 45, batches of
3 and 70), and the 5,000-item workload (r = 50) through the batch path,
the codes entry point and the server."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1807_08692_amd import workload as W

pytestmark = pytest.mark.gpu

N, R, D, KY, TOPK = 1237, 37, 45, 7, 10


def e4m3_value(code):
    """OCP FP8 E4M3 value of each code (sign, exponent bias 7, 3 mantissa
    bits, exponent field 0 = subnormals m 2^-9)."""
    code = np.asarray(code, np.int64)
    s = np.where(code & 0x80, -1.0, 1.0)
    e = (code >> 3) & 15
    m = code & 7
    return s * np.where(e == 0, m * 2.0 ** -9, 2.0 ** (e - 7.0) * (1.0 + m / 8.0))


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


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def ragged(torch_dev):
    from paper_1807_08692_amd import hd
    rng = np.random.default_rng(1237)
    rowptr, col, w = random_graph(N, 5, 3)
    s32 = O.normalize(N, rowptr, col, w.astype(np.float64)).astype(np.float32)
    g = O.Graph64.from_csr(N, rowptr, col, s32)
    U = np.linalg.qr(rng.standard_normal((N, R)))[0].astype(np.float32)
    lam = np.sort(rng.uniform(0.0, 0.95, size=R))[::-1].copy()
    V = rng.standard_normal((N, D)).astype(np.float32)
    V /= np.linalg.norm(V, axis=1, keepdims=True)
    uc, us = hd.quantize_fp8(U, True)
    vc, vs = hd.quantize_fp8(V, False)
    return dict(rowptr=rowptr, col=col, s32=s32, g=g, U=U, lam=lam, V=V, uc=uc, us=us, vc=vc, vs=vs,
                U8=e4m3_value(uc) * us.astype(np.float64)[None, :],
                V8=e4m3_value(vc) * vs.astype(np.float64)[:, None])


@pytest.mark.parametrize("B", [3, 70])
def test_ragged_fp8_parity(ragged, torch_dev, B):
    import torch
    from paper_1807_08692_amd import hd
    st = ragged
    rng = np.random.default_rng(B)
    Q = rng.standard_normal((B, D)).astype(np.float32)
    Q /= np.linalg.norm(Q, axis=1, keepdims=True)
    ctx = hd.Context(0)
    try:
        ctx.load_graph(N, st["rowptr"], st["col"], st["s32"])
        ctx.load_eigs_fp8(st["uc"], st["us"], st["lam"])
        ctx.load_descriptors(st["V"], dtype="fp8")
        q = torch.from_numpy(Q).to(torch_dev)
        out = ctx.query_batch(q, alpha=0.99, tol=0.0, max_iter=6, rank_r=-1, k_y=KY, top_k=TOPK,
                              want_x=True, want_y=True)
        torch.cuda.synchronize()
        for b in range(B):
            yi = out["y_ids"][b].cpu().numpy()
            yv = out["y_val"][b].cpu().numpy()
            s = st["V8"] @ Q[b].astype(np.float64)
            kth = np.sort(s)[::-1][KY - 1]
            assert len(set(yi.tolist())) == KY
            assert np.all(s[yi] >= kth - 1e-5), b
            assert set(np.nonzero(s > kth + 1e-5)[0].tolist()) <= set(yi.tolist()), b
            # y values are the cubes of the GPU's similarities of the dequantized rows
            assert np.allclose(yv, np.maximum(s[yi], 0) ** 3, rtol=1e-3, atol=1e-9)
            xo, *_ = O.iterate(st["g"], st["U8"], st["lam"], 0.99, yi, yv, 6, 0.0)
            x = out["x"][b].double().cpu().numpy()
            err = rel(x, xo)
            assert err <= 1e-4, (b, err)
            oid, _ = O.rank(x, TOPK)
            assert np.array_equal(out["rank_ids"][b].cpu().numpy(), oid), b
    finally:
        ctx.close()


@pytest.fixture(scope="module")
def fx():
    return W.build_fixture(W.CONFIGS["n5k"], n_queries=70, prefer_gpu=False)


def oracle_y(fx, qs):
    ids, vals = [], []
    for q in qs:
        i, v = O.observation(fx.V, q, fx.cfg.k_y)
        ids.append(i)
        vals.append(v)
    return np.stack(ids).astype(np.int32), np.stack(vals).astype(np.float32)


def test_fp8_workload_parity_and_effect(fx, torch_dev):
    import torch
    from paper_1807_08692_amd import hd
    g = O.Graph64.from_csr(fx.n, fx.rowptr, fx.col, fx.s)
    ids, vals = oracle_y(fx, fx.Q[:65])
    ti, tv = torch.from_numpy(ids).to(torch_dev), torch.from_numpy(vals).to(torch_dev)
    uc, us = hd.quantize_fp8(fx.U, True)
    U8 = e4m3_value(uc) * us.astype(np.float64)[None, :]
    kw = dict(alpha=0.99, tol=0.0, max_iter=8, rank_r=-1, k_y=fx.cfg.k_y, top_k=100, want_x=True)
    a = hd.Context(0)
    b = hd.Context(0)
    try:
        a.load_graph(fx.n, fx.rowptr, fx.col, fx.s)
        b.load_graph(fx.n, fx.rowptr, fx.col, fx.s)
        a.load_eigs(fx.U, fx.lam, dtype="fp8")      # quantized by the library
        b.load_eigs_fp8(uc, us, fx.lam)              # the same codes given
        oa = a.query_batch(None, ti, tv, **kw)
        ob = b.query_batch(None, ti, tv, **kw)
        torch.cuda.synchronize()
        xa, xb = oa["x"].cpu().numpy(), ob["x"].cpu().numpy()
        assert np.array_equal(xa, xb)
        worst_fp32 = 0.0
        for q in (0, 1, 31, 64):
            xo, *_ = O.iterate(g, U8, fx.lam, 0.99, ids[q], vals[q], 8, 0.0)
            assert rel(xa[q].astype(np.float64), xo) <= 1e-4, q
            # the storage rounding's effect against the fp32 U1 (reported)
            x32, *_ = O.iterate(g, fx.U, fx.lam, 0.99, ids[q], vals[q], 8, 0.0)
            worst_fp32 = max(worst_fp32, rel(xo, x32))
        print(f"fp8 U1 against fp32 U1 after 8 products: max rel err {worst_fp32:.3e}")
        assert worst_fp32 <= 0.2
    finally:
        a.close()
        b.close()


def test_fp8_server_matches_batch(fx, torch_dev):
    import torch
    from paper_1807_08692_amd import hd
    c = hd.Context(0)
    try:
        c.load_graph(fx.n, fx.rowptr, fx.col, fx.s)
        c.load_eigs(fx.U, fx.lam, dtype="fp8")
        c.load_descriptors(fx.V, dtype="fp8")
        kw = dict(alpha=0.99, max_iter=20, tol=1e-6, rank_r=50, k_y=fx.cfg.k_y, top_k=50)
        srv = hd.Server(c, 8, **kw)
        tk = srv.submit(q_desc=fx.Q[:6])
        res = {}
        for _ in range(100):
            if len(res) >= 6:
                break
            srv.step(1)
            got = srv.poll()
            for k, t in enumerate(got["tickets"]):
                res[int(t)] = {key: got[key][k] for key in ("ids", "scores", "iters")}
        srv.close()
        out = c.query_batch(torch.from_numpy(fx.Q[:6]).to(torch_dev), **kw)
        torch.cuda.synchronize()
        for q in range(6):
            r = res[int(tk[q])]
            assert r["iters"] == out["iters"][q]
            assert np.allclose(r["scores"], out["rank_scores"].cpu().numpy()[q], rtol=1e-5, atol=1e-12)
    finally:
        c.close()
