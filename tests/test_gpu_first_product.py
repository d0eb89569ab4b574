"""GPU parity of the first CG iteration's special cases, on a graph whose
rows have about 80 neighbours (more than one 64-edge chunk per row) and a y
whose ids repeat within a column:

  * the first sparse product gathers only the rows in the y row mask, and
    with Zs = P also skips the own-row load of the other rows;
  * y^T y comes from the y ids, counting a repeated id once with its summed
    value (as the oracle's dense y does);
  * the last iteration updates x alone.

x after 1 and 3 iterations, and the reported relative residual, are checked
against the oracle for plain CG (r = 0, Zs = P), the fp32 hybrid (Zs =
P + alpha U1 C) and the two-term bf16 hybrid (correction after the product).
Inputs are seeded and synthetic: a random symmetric graph, an orthonormal
U1 (QR of a Gaussian matrix) with eigenvalues in [0, 0.95)."""
import numpy as np
import pytest

from oracle import oracle as O

pytestmark = pytest.mark.gpu

N, R, KY = 2000, 20, 12


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
    rng = np.random.default_rng(80)
    rowptr, col, w = random_graph(N, 40, 9)
    assert np.diff(rowptr).max() > 64
    s32 = O.normalize(N, rowptr, col, w.astype(np.float64)).astype(np.float32)
    g = O.Graph64.from_csr(N, rowptr, col, s32)
    U = np.linalg.qr(rng.standard_normal((N, R)))[0].astype(np.float32)
    lam = np.sort(rng.uniform(0.0, 0.95, size=R))[::-1].copy()
    ids = np.stack([rng.choice(N, KY, replace=False) for _ in range(3)]).astype(np.int32)
    ids[0, 1] = ids[0, 0]
    ids[0, 5] = ids[0, 0]
    ids[2, 7] = ids[2, 2]
    vals = rng.uniform(0.1, 1.0, size=(3, KY)).astype(np.float32)
    hi = bf16_round(U)
    lo = bf16_round((U - hi).astype(np.float32))
    return dict(rowptr=rowptr, col=col, s32=s32, g=g, U=U, lam=lam, ids=ids, vals=vals,
                U2=hi.astype(np.float64) + lo.astype(np.float64))


@pytest.mark.parametrize("form", ["f32", "bf16x2"])
@pytest.mark.parametrize("rank_r", [0, -1])
@pytest.mark.parametrize("iters", [1, 3])
def test_first_product_and_norm(setup, form, rank_r, iters):
    import torch
    from paper_1807_08692_amd import hd
    st = setup
    dev = torch.device("cuda:0")
    ctx = hd.Context(0)
    try:
        ctx.load_graph(N, st["rowptr"], st["col"], st["s32"])
        ctx.load_eigs(st["U"], st["lam"], dtype=form)
        yi = torch.from_numpy(st["ids"]).to(dev)
        yv = torch.from_numpy(st["vals"]).to(dev)
        out = ctx.query_batch(None, yi, yv, alpha=0.99, max_iter=iters, tol=0.0, rank_r=rank_r, k_y=KY,
                              top_k=5, want_x=True)
        torch.cuda.synchronize()
        U_ = None if rank_r == 0 else (st["U2"] if form == "bf16x2" else st["U"])
        lam_ = None if rank_r == 0 else st["lam"]
        for b in range(3):
            xo, _, _, it, rr, _ = O.iterate(st["g"], U_, lam_, 0.99, st["ids"][b], st["vals"][b], iters, 0.0)
            x = out["x"][b].double().cpu().numpy()
            err = np.linalg.norm(x - xo) / np.linalg.norm(xo)
            assert err <= 1e-4, (b, err)
            assert int(out["iters"][b]) == it == iters
            assert abs(out["relres"][b] - rr) <= 1e-3 * rr, (b, out["relres"][b], rr)
    finally:
        ctx.close()
