"""Input preparation at sizes past 32-bit indexing: the workload's
eigensolver hands the vendor routines (sparse x dense products, QR, GEMM)
blocks of fewer than 2^31 elements, and its chunked form gives the same
eigenpairs as ARPACK when the chunks are forced small (TSQR, column blocks
of the sparse products, row blocks of the Gram matrices and rotations)."""
import numpy as np
import pytest

from paper_1807_08692_amd import workload as W


def test_chunks_cover_and_stay_under_the_limit():
    for n, m in ((2_000_000, 1250), (1_000_000, 1250), (2_000_000, 5000), (7, 3)):
        for chunks, width in ((W._col_chunks(n, m, W._LIB_ELEMS), lambda a, b: n * (b - a)),
                              (W._row_chunks(n, m, W._LIB_ELEMS), lambda a, b: m * (b - a))):
            assert chunks[0][0] == 0
            assert all(chunks[k][1] == chunks[k + 1][0] for k in range(len(chunks) - 1))
            assert all(width(a, b) <= W._LIB_ELEMS for a, b in chunks)
        assert W._col_chunks(n, m, W._LIB_ELEMS)[-1][1] == m
        assert W._row_chunks(n, m, W._LIB_ELEMS)[-1][1] == n
    # the block that crossed the limit: 2M items, r = 1000 plus a guard of 250
    assert 2_000_000 * 1250 > W._LIB_ELEMS


@pytest.mark.parametrize("limit", [W._LIB_ELEMS, 5000 * 7, 2000])
def test_chunked_eigensolver_matches_arpack(limit):
    fx = W.build_fixture(W.CONFIGS["n5k"], n_queries=1, r=0, prefer_gpu=False)
    s64 = fx.s.astype(np.float64)
    U0, l0, _ = W.top_eigs_arpack(fx.n, fx.rowptr, fx.col, s64, 20, 3)
    U, lam, res = W.top_eigs_chebyshev(fx.n, fx.rowptr, fx.col, s64, 20, 3, guard=12, prefer_gpu=False,
                                       tol=1e-10, max_outer=200, time_budget=60, lib_elems=limit)
    assert np.abs(lam - l0).max() <= 1e-12
    assert res.max() <= 1e-9
    # the same invariant subspace: every principal angle's cosine is 1
    assert np.linalg.svd(U0.T @ U, compute_uv=False).min() >= 1 - 1e-10


@pytest.mark.parametrize("limit", [W._LIB_ELEMS, 2000])
def test_cholqr3_orthonormal_basis_of_the_same_span(limit):
    """The eigensolver's orthogonalisation (shifted CholeskyQR3, row-chunked):
    orthonormal columns spanning the input's columns, for a well-conditioned
    block, one with condition number 1e10, and a rank-deficient one (a
    repeated column: the factorisation may fail and fall back to QR)."""
    import torch
    rng = np.random.default_rng(11)
    n, m = 3000, 40
    A = rng.standard_normal((n, m))
    Uq, _ = np.linalg.qr(rng.standard_normal((n, m)))
    Vq, _ = np.linalg.qr(rng.standard_normal((m, m)))
    ill = (Uq * np.logspace(0, -10, m)) @ Vq.T
    dup = A.copy()
    dup[:, 7] = dup[:, 3]
    for X, orth_tol in ((A, 1e-13), (ill, 1e-11), (dup, 1e-11)):
        Q = W._orth_cholqr3(torch.from_numpy(X), limit).numpy()
        assert np.abs(Q.T @ Q - np.eye(m)).max() <= orth_tol
        # every column of X lies in span(Q)
        assert np.linalg.norm(X - Q @ (Q.T @ X)) <= 1e-9 * np.linalg.norm(X)
