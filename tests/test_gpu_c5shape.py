"""GPU parity at the space-time sweep's shape: two million items, d = 512
bfloat16 descriptors, a batch of 1024 queries (solver width 1024, so one
solver vector holds N x 1024 = 2.05e9 floats, close to 2^31), about 28
entries per row, r = 100 bfloat16 eigenvector columns, autotuned launch
parameters. Sampled columns of the hybrid and of plain CG are checked against
the oracle run on the same y for the same number of products, the neighbour
selection against FP64 cosines of the rounded descriptors, and the ranking
against the oracle's sort of the GPU's x. The inputs are synthetic and cheap
to build, as in the full-size test at one million items: a random symmetric
graph, unit descriptors with independent normal entries, and an orthonormal
U1 whose columns have disjoint supports."""
import numpy as np
import pytest

from oracle import oracle as O

pytestmark = pytest.mark.gpu

N, D, R, B, KY = 2_000_000, 512, 100, 1024, 50


def bf16_round(a):
    u = np.ascontiguousarray(a, np.float32).view(np.uint32).astype(np.uint64)
    h = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint32)
    return (h << 16).view(np.float32)


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


@pytest.fixture(scope="module")
def setup():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rng = np.random.default_rng(2025)
    rowptr, col, w = random_graph(N, 14, 12)
    s64 = O.normalize(N, rowptr, col, w.astype(np.float64))
    s32 = s64.astype(np.float32)
    g = O.Graph64.from_csr(N, rowptr, col, s32)
    comp = rng.permutation(N) % R
    vals = rng.standard_normal(N).astype(np.float64)
    norms = np.zeros(R)
    np.add.at(norms, comp, vals ** 2)
    vals /= np.sqrt(norms[comp])
    U = np.zeros((N, R), np.float32)
    U[np.arange(N), comp] = vals.astype(np.float32)
    lam = np.sort(rng.uniform(0.0, 0.95, size=R))[::-1].copy()
    V = rng.standard_normal((N, D), dtype=np.float32)
    V /= np.linalg.norm(V, axis=1, keepdims=True)
    Q = rng.standard_normal((B, D), dtype=np.float32)
    Q /= np.linalg.norm(Q, axis=1, keepdims=True)
    return dict(rowptr=rowptr, col=col, s32=s32, g=g, U=U, lam=lam, V=V, Q=Q, comp=comp, vals=vals)


def test_c5_shape_parity(setup):
    import torch
    from paper_1807_08692_amd import hd
    dev = torch.device("cuda:0")
    st = setup
    print(f"[c5 shape] N={N} B={B} r={R} nnz={st['col'].size}", flush=True)
    ctx = hd.Context(0)
    try:
        ctx.load_graph(N, st["rowptr"], st["col"], st["s32"])
        ctx.load_eigs(st["U"], st["lam"], dtype="bf16")
        ctx.load_descriptors(st["V"], dtype="bf16")
        tune = ctx.autotune(B, 2)
        q = torch.from_numpy(st["Q"]).to(dev)
        kw = dict(alpha=0.99, tol=0.0, k_y=KY, top_k=100, want_y=True)
        hyb = ctx.query_batch(q, max_iter=5, rank_r=-1, want_x=True, **kw)
        torch.cuda.synchronize()
        hx = {b: hyb["x"][b].double().cpu().numpy() for b in (0, 700, B - 1)}
        del hyb["x"]
        pl = ctx.query_batch(q, max_iter=8, rank_r=0, want_x=True, **kw)
        torch.cuda.synchronize()
        px = {b: pl["x"][b].double().cpu().numpy() for b in (0, 700, B - 1)}
        del pl["x"]
        U1 = np.zeros((N, R))
        U1[np.arange(N), st["comp"]] = bf16_round(st["vals"].astype(np.float32)).astype(np.float64)
        for b in (0, 700, B - 1):
            yi = hyb["y_ids"][b].cpu().numpy()
            yv = hyb["y_val"][b].cpu().numpy()
            if b == 0:
                s = bf16_round(st["V"]).astype(np.float64) @ st["Q"][b].astype(np.float64)
                kth = np.sort(s)[::-1][KY - 1]
                assert np.all(s[yi] >= kth - 1e-5)
                assert set(np.nonzero(s > kth + 1e-5)[0].tolist()) <= set(yi.tolist())
            assert np.array_equal(pl["y_ids"][b].cpu().numpy(), yi)
            for out, xg, U_, lam_, it in ((hyb, hx, U1, st["lam"], 5), (pl, px, None, None, 8)):
                xo, *_ = O.iterate(st["g"], U_, lam_, 0.99, yi, yv, it, 0.0)
                x = xg[b]
                err = np.linalg.norm(x - xo) / np.linalg.norm(xo)
                assert err <= 1e-4, (b, it, err, tune)
                oid, _ = O.rank(x, 100)
                assert np.array_equal(out["rank_ids"][b].cpu().numpy(), oid)
            print(f"[c5 shape] column {b} checked", flush=True)
    finally:
        ctx.close()
