"""CPU tests of the (r, i) planner (hd_rank_plan, host-only library code):
the iteration counts it returns must achieve the A-norm accuracy the CG bound
of Section 5 promises, checked on the FP64 oracle's CG on small graphs with
the full spectrum known, and the cost model must pick the cheapest
candidate."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1807_08692_amd import hd
from paper_1807_08692_amd import workload as W

ALPHA = 0.99


def graph(seed, n=160, d=16, clusters=6, kappa=12.0, k=8):
    V, _, _ = W.vmf_mixture(n, d, clusters, kappa, seed, seed + 1)
    nbr, sim = W.knn_lists(V, k, prefer_gpu=False)
    rowptr, col, w = W.mutual_knn_graph(nbr, sim, n)
    s = O.normalize(n, rowptr, col, w)
    return O.Graph64.from_csr(n, rowptr, col, s)


@pytest.mark.parametrize("seed", [31, 57])
@pytest.mark.parametrize("eps", [1e-2, 1e-4, 1e-8])
def test_planned_iterations_reach_eps_in_a_norm(seed, eps):
    g = graph(seed)
    S = g.dense()
    w, Uf = np.linalg.eigh(S)
    o = np.argsort(-w)
    w, Uf = w[o], Uf[:, o]
    cands = [0, 1, 3, 10, 40]
    # planner given only the 60 leading eigenvalues and the exact lambda_min
    plan = hd.rank_plan(w[:60], cands, alpha=ALPHA, eps=eps, lambda_min=w[-1])
    rng = np.random.default_rng(seed)
    for c, r in enumerate(cands):
        it = int(plan["iters"][c])
        assert 1 <= it < 10000
        U, lam = Uf[:, :r], w[:r]
        A = (np.eye(g.n) - ALPHA * (S - (U * lam) @ U.T)) / (1 - ALPHA)
        for t in range(3):
            ids = np.sort(rng.choice(g.n, size=5, replace=False)).astype(np.int32)
            y = O.dense_y(g.n, ids, rng.uniform(0.1, 1.0, size=5))
            xstar = np.linalg.solve(A, y)
            xi, _, _, _ = O.cg(g, U if r else None, lam, ALPHA, y, it, 0.0)
            e = xstar - xi
            rel = np.sqrt(max(e @ A @ e, 0.0)) / np.sqrt(xstar @ A @ xstar)
            assert rel <= eps * (1 + 1e-6) + 1e-13, (r, it, rel)


def test_outlier_refinement_beats_plain_bound_for_r0():
    """With lambda_1 = 1 above a gap, the plain bound of eq. (bound) with
    k from eq. (cond-r) at r = 0 needs far more iterations than the refined
    count; the refined count is still guaranteed (previous test)."""
    lam = np.r_[1.0, np.linspace(0.32, 0.29, 99)]
    plan = hd.rank_plan(lam, [0, 1], alpha=ALPHA, eps=1e-3, lambda_min=-1.0)
    k0 = (1 + ALPHA) / (1 - ALPHA)
    q0 = (np.sqrt(k0) - 1) / (np.sqrt(k0) + 1)
    plain = int(np.ceil(np.log(2 / 1e-3) / np.log(1 / q0)))
    assert plan["iters"][0] < plain // 3
    assert plan["iters"][1] < plan["iters"][0]


def test_cost_model_picks_cheapest():
    lam = np.r_[1.0, np.linspace(0.6, 0.1, 199)]
    cands = [0, 32, 100, 200]
    fixed = np.array([10.0, 11.0, 12.0, 14.0])
    per_it = np.array([9.0, 9.5, 11.0, 13.0])
    plan = hd.rank_plan(lam, cands, alpha=ALPHA, eps=1e-3, lambda_min=-1.0, fixed_ms=fixed, iter_ms=per_it)
    pred = fixed + plan["iters"] * per_it
    assert np.allclose(plan["pred_ms"], pred)
    assert plan["best"] == int(np.argmin(pred))


def test_rejects_bad_arguments():
    with pytest.raises(hd.HDError):
        hd.rank_plan([0.5, 0.9], [0], eps=1e-3)          # not descending
    with pytest.raises(hd.HDError):
        hd.rank_plan([0.9, 0.5], [3], eps=1e-3)          # r beyond the spectrum
    with pytest.raises(hd.HDError):
        hd.rank_plan([0.9, 0.5], [0], eps=0.0)
