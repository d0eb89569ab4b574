"""GPU parity on large random sparse symmetric graphs (P of 179 MB and
205 MB, more than the Infinity Cache holds), with the library normalising W
itself (HD_GRAPH_NORMALIZE) against the oracle's normalisation. A few
sampled query columns are checked against the oracle's CG run for the same
number of products."""
import numpy as np
import pytest

from oracle import oracle as O

pytestmark = pytest.mark.gpu


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


@pytest.mark.parametrize("n,B", [(700_000, 64), (200_000, 256)])
def test_large_graph_parity(n, B):
    import torch
    from paper_1807_08692_amd import hd
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dev = torch.device("cuda:0")
    rowptr, col, w = random_graph(n, 5, n + B)
    s_oracle = O.normalize(n, rowptr, col, w.astype(np.float64))
    g = O.Graph64.from_csr(n, rowptr, col, s_oracle.astype(np.float32))
    rng = np.random.default_rng(7)
    ky = 10
    ids = np.stack([rng.choice(n, size=ky, replace=False) for _ in range(B)]).astype(np.int32)
    vals = rng.uniform(0.1, 1.0, size=(B, ky)).astype(np.float32)
    with hd.Context(0) as ctx:
        ctx.load_graph(n, rowptr, col, w, normalize=True)
        out = ctx.query_batch(None, torch.from_numpy(ids).to(dev), torch.from_numpy(vals).to(dev),
                              alpha=0.99, max_iter=4, tol=0.0, rank_r=0, k_y=ky, top_k=10, want_x=True)
        torch.cuda.synchronize()
    x = out["x"].cpu().numpy()
    for b in (0, B // 2 + 3, B - 1):
        assert out["iters"][b] == 4
        xo, *_ = O.iterate(g, None, None, 0.99, ids[b], vals[b], 4, 0.0)
        err = np.linalg.norm(x[b] - xo) / np.linalg.norm(xo)
        assert err <= 1e-4, (b, err)
