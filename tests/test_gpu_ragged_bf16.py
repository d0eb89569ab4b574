"""GPU parity of the bfloat16 forms where every stored operand is padded:
N = 1237 items (the last 16-item operand tile holds 5), r = 37 eigenvectors
(rounded up to 64 components), d = 45 descriptor dimensions (rounded up to
64) and batches of 3 and 70 queries (query tiles padded to 64 rows). The
bfloat16 kernels read their operands in 16 x 32 tiles, so each padding is
read and must contribute nothing.

Checks per query: the neighbour set against FP64 cosines of the rounded
descriptors, x against the oracle run on the GPU's own y with the two-term
U1 as stored (hi + lo), and the ranking against the oracle's sort of the
GPU's x. Inputs are seeded and synthetic: a random symmetric graph with
about ten neighbours per item, an orthonormal U1 (QR of a Gaussian matrix),
eigenvalues in [0, 0.95) and unit descriptors."""
import numpy as np
import pytest

from oracle import oracle as O

pytestmark = pytest.mark.gpu

N, R, D, KY, TOPK = 1237, 37, 45, 7, 10


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
    rng = np.random.default_rng(1237)
    rowptr, col, w = random_graph(N, 5, 3)
    s32 = O.normalize(N, rowptr, col, w.astype(np.float64)).astype(np.float32)
    g = O.Graph64.from_csr(N, rowptr, col, s32)
    U = np.linalg.qr(rng.standard_normal((N, R)))[0].astype(np.float32)
    lam = np.sort(rng.uniform(0.0, 0.95, size=R))[::-1].copy()
    V = rng.standard_normal((N, D)).astype(np.float32)
    V /= np.linalg.norm(V, axis=1, keepdims=True)
    hi = bf16_round(U)
    lo = bf16_round((U - hi).astype(np.float32))
    U2 = hi.astype(np.float64) + lo.astype(np.float64)
    return dict(rowptr=rowptr, col=col, s32=s32, g=g, U=U, U2=U2, lam=lam, V=V,
                Vr=bf16_round(V).astype(np.float64), rng=rng)


@pytest.mark.parametrize("B", [3, 70])
def test_ragged_bf16_parity(setup, B):
    import torch
    from paper_1807_08692_amd import hd
    st = setup
    rng = np.random.default_rng(B)
    Q = rng.standard_normal((B, D)).astype(np.float32)
    Q /= np.linalg.norm(Q, axis=1, keepdims=True)
    ctx = hd.Context(0)
    try:
        ctx.load_graph(N, st["rowptr"], st["col"], st["s32"])
        ctx.load_eigs(st["U"], st["lam"], dtype="bf16x2")
        ctx.load_descriptors(st["V"], dtype="bf16")
        q = torch.from_numpy(Q).to(torch.device("cuda:0"))
        out = ctx.query_batch(q, alpha=0.99, tol=0.0, max_iter=6, rank_r=-1, k_y=KY, top_k=TOPK,
                              want_x=True, want_y=True)
        torch.cuda.synchronize()
        for b in range(B):
            yi = out["y_ids"][b].cpu().numpy()
            yv = out["y_val"][b].cpu().numpy()
            s = st["Vr"] @ Q[b].astype(np.float64)
            kth = np.sort(s)[::-1][KY - 1]
            assert len(set(yi.tolist())) == KY
            assert np.all(s[yi] >= kth - 1e-5), b
            assert set(np.nonzero(s > kth + 1e-5)[0].tolist()) <= set(yi.tolist()), b
            xo, *_ = O.iterate(st["g"], st["U2"], st["lam"], 0.99, yi, yv, 6, 0.0)
            x = out["x"][b].double().cpu().numpy()
            err = np.linalg.norm(x - xo) / np.linalg.norm(xo)
            assert err <= 1e-4, (b, err)
            oid, _ = O.rank(x, TOPK)
            assert np.array_equal(out["rank_ids"][b].cpu().numpy(), oid), b
    finally:
        ctx.close()
