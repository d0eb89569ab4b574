"""GPU parity of general filters (Appendix A): x = h(S) y for a polynomial h
(a truncated heat kernel and a random polynomial), computed as the spectral
term with g = h - h(0) plus h(S_r) y by Horner's rule on the deflated
operator, against the oracle's term-by-term sum with the same stored U1
(fp32, two-term bf16, sparsified)."""
from math import exp, factorial

import numpy as np
import pytest

from oracle import oracle as O
from paper_1807_08692_amd import workload as W

pytestmark = pytest.mark.gpu


def bf16_round(a):
    u = np.ascontiguousarray(a, np.float32).view(np.uint32).astype(np.uint64)
    h = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint32)
    return (h << 16).view(np.float32)


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def fx():
    return W.build_fixture(W.CONFIGS["n5k"], n_queries=200, prefer_gpu=False)


@pytest.fixture(scope="module")
def g64(fx):
    return O.Graph64.from_csr(fx.n, fx.rowptr, fx.col, fx.s)


def stored_u(fx, form):
    if form == "f32":
        return fx.U.astype(np.float64)
    if form == "bf16x2":
        hi = bf16_round(fx.U)
        lo = bf16_round((fx.U - hi).astype(np.float32))
        return hi.astype(np.float64) + lo.astype(np.float64)
    rp, col, val = W.sparsify_eigvecs(fx.U, 0.9)
    return W.sparse_to_dense(fx.n, fx.U.shape[1], rp, col, val)


HEAT = [exp(-5.0) * 5.0 ** i / factorial(i) for i in range(26)]
POLY = list(np.random.default_rng(9).uniform(-0.5, 0.5, size=9))


@pytest.mark.parametrize("form", ["f32", "bf16x2", "sparse90"])
@pytest.mark.parametrize("coeffs", [HEAT, POLY], ids=["heat", "poly"])
@pytest.mark.parametrize("B,r_use", [(3, -1), (70, 0), (130, 20)])
def test_filter_parity(fx, g64, torch_dev, form, coeffs, B, r_use):
    import torch
    from paper_1807_08692_amd import hd
    r = fx.U.shape[1]
    c = hd.Context(0)
    try:
        c.load_graph(fx.n, fx.rowptr, fx.col, fx.s)
        if form == "sparse90":
            rp, col, val = W.sparsify_eigvecs(fx.U, 0.9)
            c.load_eigs_sparse(r, rp, col, val, fx.lam)
        else:
            c.load_eigs(fx.U, fx.lam, dtype=form)
        Us = stored_u(fx, form)
        ids, vals = [], []
        for q in fx.Q[:B]:
            i, v = O.observation(fx.V, q, fx.cfg.k_y)
            ids.append(i)
            vals.append(v)
        ids = np.stack(ids).astype(np.int32)
        vals = np.stack(vals).astype(np.float32)
        out = c.query_filter(coeffs, None, torch.from_numpy(ids).to(torch_dev),
                             torch.from_numpy(vals).to(torch_dev), rank_r=r_use, top_k=50, want_x=True)
        torch.cuda.synchronize()
        x = out["x"].cpu().numpy()
        ru = r if r_use < 0 else r_use
        for b in sorted({0, B // 2, B - 1}):
            xo = O.filter_poly(g64, Us[:, :ru] if ru else None, fx.lam[:ru], coeffs, ids[b], vals[b])
            err = np.linalg.norm(x[b] - xo) / np.linalg.norm(xo)
            assert err <= 1e-4, (b, err)
            oid, _ = O.rank(x[b].astype(np.float64), 50)
            assert np.array_equal(out["rank_ids"].cpu().numpy()[b], oid)
    finally:
        c.close()


def test_filter_rejects_bad_coefficients(fx, torch_dev):
    import torch
    from paper_1807_08692_amd import hd
    c = hd.Context(0)
    try:
        c.load_graph(fx.n, fx.rowptr, fx.col, fx.s)
        q = torch.from_numpy(fx.Q[:2]).to(torch_dev)
        c.load_descriptors(fx.V)
        with pytest.raises(hd.HDError):
            c.query_filter([1.0, float("nan")], q, k_y=10)
    finally:
        c.close()
