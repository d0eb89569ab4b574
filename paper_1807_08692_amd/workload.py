"""Seeded synthetic workloads: database descriptors, queries, the k-NN graph
and its leading eigenpairs.

This module only prepares inputs. It holds none of the query-time arithmetic
(the observation vector, the spectral term, the conjugate-gradient solve and
the ranking live in the HIP library, and separately in the FP64 oracle).
What it builds is the off-line side of Section 3 and Section 6.1 of Iscen et
al. (the database, its reciprocal k-NN graph with (v^T z)_+^3 weights, the
symmetric normalisation, and the r leading eigenpairs that the hybrid method
assumes were computed off-line), on synthetic data in place of the paper's
image descriptors:

* descriptors: a mixture of von Mises-Fisher distributions on the unit
  sphere S^(d-1), cluster centres uniform on the sphere, each point drawn
  from vMF(mu_c, kappa) by Wood's rejection sampler (Wood 1994,
  "Simulation of the von Mises Fisher distribution");
* queries: further draws from the same mixture with an independent stream;
* graph: mutual ("reciprocal") k-NN over cosine similarity, self excluded,
  weight max(0, cos)^3, zero diagonal, then D^-1/2 W D^-1/2;
* eigenpairs: the r algebraically largest eigenpairs of the normalised
  graph, from ARPACK (small graphs) or a Chebyshev-filtered subspace
  iteration (large graphs, torch on the GPU when one is present).

Everything is deterministic given the seed. Bulk similarity products and the
large eigensolve use torch on the GPU when available: this is input
preparation outside the library, and its results are handed to both the
library and the oracle as plain arrays.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field
from typing import Optional

import numpy as np


# --------------------------------------------------------------------------
# Configurations (shapes of the paper's large-scale setting, Section 6.1:
# alpha = 0.99, reciprocal k-NN, d = 2048 descriptors)
# --------------------------------------------------------------------------

@dataclass(frozen=True)
class WorkloadConfig:
    name: str
    n: int
    d: int
    clusters: int
    kappa: float
    k: int                 # neighbours per item in the reciprocal k-NN graph
    alpha: float
    r: int                 # rank of the spectral term
    batch: int             # queries per batch
    k_y: int               # non-zeros of the observation vector
    tol: float             # CG stopping rule on the relative residual
    max_iter: int
    seed_base: int

    @property
    def seeds(self):
        """(centres, points, queries, eigensolver start) seeds."""
        b = self.seed_base
        return b + 1, b + 2, b + 3, b + 4


CONFIGS = {
    # 5,000 items, d=128, 50 vMF clusters (kappa 40), k=10, r in {0, 50}.
    "n5k": WorkloadConfig("n5k", 5000, 128, 50, 40.0, 10, 0.99, 50, 1, 10, 1e-6, 20, 0),
    # 100,000 items, d=2048, 1,000 clusters (kappa 60), k=50, r=400, 64 queries.
    "n100k": WorkloadConfig("n100k", 100_000, 2048, 1000, 60.0, 50, 0.99, 400, 64, 50, 1e-5, 100, 1000),
    # 1,000,000 items, d=2048, 10,000 clusters (kappa 60), k=50, r=1000, 256 queries.
    "n1m": WorkloadConfig("n1m", 1_000_000, 2048, 10_000, 60.0, 50, 0.99, 1000, 256, 50, 1e-5, 100, 2000),
    # the serving configuration's two smaller resident databases (d=2048, k=50,
    # N/100 clusters): 50,000 items with r=200, 300,000 items with r=400
    "n50k": WorkloadConfig("n50k", 50_000, 2048, 500, 60.0, 50, 0.99, 200, 64, 50, 1e-5, 100, 5000),
    "n300k": WorkloadConfig("n300k", 300_000, 2048, 3000, 60.0, 50, 0.99, 400, 64, 50, 1e-5, 100, 6000),
    # 2,000,000 items, d=512, 20,000 clusters (kappa 60), k=30, r up to 4000, 1024 queries.
    "n2m": WorkloadConfig("n2m", 2_000_000, 512, 20_000, 60.0, 30, 0.99, 400, 1024, 50, 1e-3, 100, 4000),
}


# --------------------------------------------------------------------------
# von Mises-Fisher mixture (Wood 1994)
# --------------------------------------------------------------------------

def _wood_w(rng: np.random.Generator, d: int, kappa: float, m: int) -> np.ndarray:
    """m samples of w = mu^T x for x ~ vMF(mu, kappa) on S^(d-1), by Wood's
    rejection scheme (envelope from a Beta((d-1)/2, (d-1)/2) variate)."""
    dm1 = d - 1.0
    b = dm1 / (2.0 * kappa + math.sqrt(4.0 * kappa * kappa + dm1 * dm1))
    x0 = (1.0 - b) / (1.0 + b)
    c = kappa * x0 + dm1 * math.log(1.0 - x0 * x0)
    out = np.empty(m)
    filled = 0
    while filled < m:
        need = m - filled
        draw = max(16, int(need * 1.3))
        z = rng.beta(dm1 / 2.0, dm1 / 2.0, size=draw)
        u = rng.uniform(size=draw)
        w = (1.0 - (1.0 + b) * z) / (1.0 - (1.0 - b) * z)
        ok = kappa * w + dm1 * np.log(1.0 - x0 * w) - c >= np.log(u)
        acc = w[ok][:need]
        out[filled:filled + acc.size] = acc
        filled += acc.size
    return out


def vmf_draw(rng: np.random.Generator, mus: np.ndarray, kappa: float) -> np.ndarray:
    """One vMF(mu_i, kappa) draw for each row mu_i of mus (unit rows)."""
    m, d = mus.shape
    w = _wood_w(rng, d, kappa, m)
    v = rng.standard_normal((m, d))
    v -= np.sum(v * mus, axis=1, keepdims=True) * mus      # tangent direction
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    x = w[:, None] * mus + np.sqrt(np.maximum(0.0, 1.0 - w * w))[:, None] * v
    x /= np.linalg.norm(x, axis=1, keepdims=True)
    return x


def vmf_draw_torch(rng: np.random.Generator, gen, mus, kappa: float):
    """vmf_draw with the tangent Gaussians drawn by torch on mus's device
    (gen: a seeded torch.Generator on that device)."""
    import torch
    m, d = mus.shape
    w = torch.from_numpy(_wood_w(rng, d, kappa, m)).to(mus.device)
    v = torch.randn((m, d), generator=gen, device=mus.device, dtype=torch.float64)
    v -= (v * mus).sum(1, keepdim=True) * mus
    v /= torch.linalg.vector_norm(v, dim=1, keepdim=True)
    x = w[:, None] * mus + torch.sqrt(torch.clamp(1.0 - w * w, min=0.0))[:, None] * v
    return x / torch.linalg.vector_norm(x, dim=1, keepdim=True)


def vmf_mixture(n: int, d: int, clusters: int, kappa: float, seed_centres: int,
                seed_points: int, chunk: int = 65536, device=None):
    """n unit-norm float32 descriptors from an equal-weight vMF mixture.
    Returns (V n x d float32, labels n int32, centres clusters x d float64).
    With a torch GPU device the tangent Gaussians come from torch's seeded
    generator there (a different, equally deterministic stream)."""
    rc = np.random.default_rng(seed_centres)
    centres = rc.standard_normal((clusters, d))
    centres /= np.linalg.norm(centres, axis=1, keepdims=True)
    rp = np.random.default_rng(seed_points)
    labels = rp.integers(0, clusters, size=n).astype(np.int32)
    V = np.empty((n, d), np.float32)
    if device is not None:
        import torch
        gen = torch.Generator(device=device).manual_seed(int(seed_points))
        ct = torch.from_numpy(centres).to(device)
        lt = torch.from_numpy(labels.astype(np.int64)).to(device)
        for s in range(0, n, chunk):
            e = min(n, s + chunk)
            V[s:e] = vmf_draw_torch(rp, gen, ct[lt[s:e]], kappa).float().cpu().numpy()
    else:
        for s in range(0, n, chunk):
            e = min(n, s + chunk)
            V[s:e] = vmf_draw(rp, centres[labels[s:e]], kappa).astype(np.float32)
    # re-normalise in float32 so every stored row is unit norm to fp32 rounding
    V /= np.linalg.norm(V, axis=1, keepdims=True).astype(np.float32)
    return V, labels, centres


def vmf_queries(m: int, centres: np.ndarray, kappa: float, seed: int) -> np.ndarray:
    rq = np.random.default_rng(seed)
    lab = rq.integers(0, centres.shape[0], size=m)
    Q = vmf_draw(rq, centres[lab], kappa).astype(np.float32)
    Q /= np.linalg.norm(Q, axis=1, keepdims=True).astype(np.float32)
    return Q


# --------------------------------------------------------------------------
# Reciprocal k-NN graph
# --------------------------------------------------------------------------

def _torch_device(prefer_gpu: bool = True):
    import torch
    if prefer_gpu and torch.cuda.is_available():
        return torch.device("cuda:0")
    return torch.device("cpu")


def knn_lists(V: np.ndarray, k: int, prefer_gpu: bool = True, block: int = 4096,
              bf16_inputs: bool = False):
    """Per item, its k most similar other items by cosine (self excluded),
    with the float32 similarities. Returns (nbr n x k int64, sim n x k float32).
    bf16_inputs: form the products from bfloat16-rounded descriptors with
    fp32 accumulation and fp32 results (for very large n on the GPU)."""
    import torch
    dev = _torch_device(prefer_gpu)
    n = V.shape[0]
    Vt = torch.from_numpy(np.ascontiguousarray(V)).to(dev)
    Vb = Vt.to(torch.bfloat16) if (bf16_inputs and dev.type == "cuda") else None
    nbr = np.empty((n, k), np.int64)
    sim = np.empty((n, k), np.float32)
    if dev.type == "cuda":
        block = max(256, min(block, int(2 ** 31 // max(n, 1))))

    def products(s, e):
        if Vb is not None:
            try:
                return torch.mm(Vb[s:e], Vb.T, out_dtype=torch.float32)
            except (TypeError, RuntimeError, NotImplementedError):
                pass
        return Vt[s:e] @ Vt.T

    for s in range(0, n, block):
        e = min(n, s + block)
        S = products(s, e)
        S[torch.arange(e - s, device=dev), torch.arange(s, e, device=dev)] = -float("inf")
        val, idx = torch.topk(S, k, dim=1, largest=True, sorted=True)
        nbr[s:e] = idx.cpu().numpy()
        sim[s:e] = val.cpu().numpy()
        del S
    return nbr, sim


def mutual_knn_graph(nbr: np.ndarray, sim: np.ndarray, n: int):
    """Reciprocal k-NN adjacency W (Section 6.1): edge i-j iff each is among
    the other's k nearest neighbours; weight max(0, cos)^3, zero diagonal,
    edges of weight 0 dropped. The cosine of an edge is taken from its
    lower-id endpoint's list so W is exactly symmetric.
    Returns CSR (rowptr int64[n+1], col int32[nnz], w float64[nnz])."""
    k = nbr.shape[1]
    rows = np.repeat(np.arange(n, dtype=np.int64), k)
    cols = nbr.reshape(-1)
    vals = sim.reshape(-1).astype(np.float64)
    key = rows * n + cols
    rkey = cols * n + rows
    order = np.argsort(key, kind="stable")
    skey = key[order]
    pos = np.searchsorted(skey, rkey)
    pos = np.minimum(pos, skey.size - 1)
    mutual = skey[pos] == rkey
    # canonical similarity: from the (min, max) orientation
    other = vals[order[pos]]
    canon = np.where(rows < cols, vals, other)
    rows, cols, canon = rows[mutual], cols[mutual], canon[mutual]
    w = np.maximum(canon, 0.0) ** 3
    keep = w > 0.0
    rows, cols, w = rows[keep], cols[keep], w[keep]
    o = np.lexsort((cols, rows))
    rows, cols, w = rows[o], cols[o], w[o]
    rowptr = np.zeros(n + 1, np.int64)
    np.add.at(rowptr, rows + 1, 1)
    rowptr = np.cumsum(rowptr)
    return rowptr, cols.astype(np.int32), w


def mutual_knn_graph_torch(nbr, sim, n: int, device):
    """mutual_knn_graph on a torch device (same result, sorted keys on the GPU)."""
    import torch
    k = nbr.shape[1]
    nb = torch.from_numpy(np.ascontiguousarray(nbr)).to(device).reshape(-1)
    sv = torch.from_numpy(np.ascontiguousarray(sim)).to(device).reshape(-1).double()
    rows = torch.arange(n, device=device, dtype=torch.int64).repeat_interleave(k)
    key = rows * n + nb
    skey, order = torch.sort(key)
    vals = sv[order]
    rs, cs = skey // n, skey % n
    rkey = cs * n + rs
    pos = torch.searchsorted(skey, rkey).clamp(max=skey.numel() - 1)
    mutual = skey[pos] == rkey
    canon = torch.where(rs < cs, vals, vals[pos])
    w = torch.clamp(canon, min=0.0) ** 3
    keep = mutual & (w > 0.0)
    rs, cs, w = rs[keep], cs[keep], w[keep]
    rowptr = torch.zeros(n + 1, dtype=torch.int64, device=device)
    rowptr[1:] = torch.cumsum(torch.bincount(rs, minlength=n), 0)
    return rowptr.cpu().numpy(), cs.to(torch.int32).cpu().numpy(), w.cpu().numpy()


def symmetric_normalize(n, rowptr, col, w):
    """Section 3: D^-1/2 W D^-1/2 on W's pattern (float64); zero-degree items
    get a zero row."""
    deg = np.zeros(n)
    rows = np.repeat(np.arange(n), np.diff(rowptr))
    np.add.at(deg, rows, w)
    dinv = np.where(deg > 0, 1.0 / np.sqrt(np.where(deg > 0, deg, 1.0)), 0.0)
    return w * (dinv[rows] * dinv[col])


# --------------------------------------------------------------------------
# Leading eigenpairs (off-line input of the hybrid method)
# --------------------------------------------------------------------------

def top_eigs_arpack(n, rowptr, col, sval, r, seed):
    """r algebraically largest eigenpairs (descending) with ARPACK."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as sla
    if r == 0:
        return np.zeros((n, 0)), np.zeros(0), np.zeros(0)
    A = sp.csr_matrix((np.asarray(sval, np.float64), col, rowptr), shape=(n, n))
    v0 = np.random.default_rng(seed).standard_normal(n)
    if r >= n - 1:
        w, Uf = np.linalg.eigh(A.toarray())
        o = np.argsort(-w, kind="stable")[:r]
        w, Uf = w[o], Uf[:, o]
    else:
        w, Uf = sla.eigsh(A, k=r, which="LA", v0=v0, tol=1e-13, maxiter=100000)
        o = np.argsort(-w, kind="stable")
        w, Uf = w[o], Uf[:, o]
    res = np.linalg.norm(A @ Uf - Uf * w, axis=0)
    return Uf, w, res


# Dense operands handed to the vendor routines below (sparse x dense
# products, QR, GEMM) stay under 2^31 elements: those routines index with
# 32-bit integers, and a 2M x 1250 double block (2.5e9 elements) is past it.
_LIB_ELEMS = (1 << 31) - 1


def _col_chunks(n, m, limit):
    w = max(1, min(m, limit // max(n, 1)))
    return [(a, min(m, a + w)) for a in range(0, m, w)]


def _row_chunks(n, m, limit):
    h = max(1, min(n, limit // max(m, 1)))
    return [(a, min(n, a + h)) for a in range(0, n, h)]


def _spmm_chunked(S, X, limit):
    """S @ X column block by column block (each block n x w, w n < limit)."""
    import torch
    n, m = X.shape
    out = torch.empty_like(X)
    for a, b in _col_chunks(n, m, limit):
        out[:, a:b] = S @ X[:, a:b].contiguous()
    return out


def _gram_chunked(A, B, limit):
    """A^T B summed over row blocks in order."""
    n, m = A.shape
    G = None
    for a, b in _row_chunks(n, max(m, B.shape[1]), limit):
        g = A[a:b].T @ B[a:b]
        G = g if G is None else G + g
    return G


def _rotate_chunked(X, Z, limit):
    """X @ Z row block by row block."""
    import torch
    n, m = X.shape
    out = torch.empty((n, Z.shape[1]), dtype=X.dtype, device=X.device)
    for a, b in _row_chunks(n, max(m, Z.shape[1]), limit):
        out[a:b] = X[a:b] @ Z
    return out


def _qr_chunked(X, limit):
    """Orthonormal basis of X's columns: one Householder QR when X is small
    enough, else TSQR (QR of each row block, QR of the stacked R factors,
    and the block Q factors times the matching slices of the second Q)."""
    import torch
    n, m = X.shape
    if n * m <= limit:
        return torch.linalg.qr(X)[0]
    blocks = _row_chunks(n, m, limit)
    Qs, Rs = [], []
    for a, b in blocks:
        q, r_ = torch.linalg.qr(X[a:b])
        Qs.append(q)
        Rs.append(r_)
    Q2, _ = torch.linalg.qr(torch.cat(Rs, dim=0))
    out = torch.empty_like(X)
    k = 0
    for (a, b), q in zip(blocks, Qs):
        w = q.shape[1]
        out[a:b] = q @ Q2[k:k + w]
        k += w
    return out


def _orth_cholqr3(X, limit):
    """Orthonormal basis of X's columns by shifted CholeskyQR3 (Fukaya,
    Kannan, Nakatsukasa, Zhang and Yamamoto, 2020): a Cholesky QR of the
    Gram matrix shifted by 11 (n m + m (m + 1)) u ||G||_F, then two plain
    Cholesky QR passes; every product over the n rows in row blocks of fewer
    than `limit` elements (the Gram matrices summed in order). Falls back to
    _qr_chunked when a Cholesky factorisation fails. One pass is three Gram
    products, three m x m factorisations and three rotations, against a
    Householder QR of the whole block (16.5 s for 1M x 1250 in FP64 on the
    device, 0.3 s this way)."""
    import torch
    n, m = X.shape
    u = float(torch.finfo(X.dtype).eps) / 2.0
    Y = X
    for p in range(3):
        G = _gram_chunked(Y, Y, limit)
        G = 0.5 * (G + G.T)
        if p == 0:
            shift = 11.0 * (n * m + m * (m + 1)) * u * float(torch.linalg.matrix_norm(G))
            G = G + shift * torch.eye(m, dtype=G.dtype, device=G.device)
        L, info = torch.linalg.cholesky_ex(G)
        if int(info) != 0:
            return _qr_chunked(X, limit)
        Rinv = torch.linalg.solve_triangular(L.T, torch.eye(m, dtype=G.dtype, device=G.device), upper=True)
        Y = _rotate_chunked(Y, Rinv, limit)
    return Y


def top_eigs_chebyshev(n, rowptr, col, sval, r, seed, guard=None, degree=12,
                       max_outer=60, tol=1e-9, time_budget=120.0, prefer_gpu=True,
                       lib_elems=_LIB_ELEMS, log=None):
    """r algebraically largest eigenpairs by Chebyshev-filtered subspace
    iteration with Rayleigh-Ritz, in float64 (torch; GPU if present).
    The filter damps the interval [-1, b] with b the smallest Ritz value of
    the block. Every sparse product, QR, Gram matrix and rotation works on
    blocks of fewer than lib_elems elements. Returns (U n x r, lambda r,
    residual norms r)."""
    import torch
    dev = _torch_device(prefer_gpu)
    if r == 0:
        return np.zeros((n, 0)), np.zeros(0), np.zeros(0)
    m = r + (guard if guard is not None else max(20, r // 4))
    m = min(m, n)
    S = torch.sparse_csr_tensor(torch.from_numpy(np.asarray(rowptr, np.int64)),
                                torch.from_numpy(np.asarray(col, np.int64)),
                                torch.from_numpy(np.asarray(sval, np.float64)),
                                size=(n, n)).to(dev)
    g = torch.Generator(device="cpu").manual_seed(int(seed))
    X = torch.randn(n, m, generator=g, dtype=torch.float64).to(dev)
    X = _orth_cholqr3(X, lib_elems)
    t0 = time.time()
    lam = None
    res = None
    for outer in range(max_outer):
        SX = _spmm_chunked(S, X, lib_elems)
        H = _gram_chunked(X, SX, lib_elems)
        H = 0.5 * (H + H.T)
        w, Z = torch.linalg.eigh(H)
        w, Z = w.flip(0), Z.flip(1)
        X = _rotate_chunked(X, Z, lib_elems)
        SX = _rotate_chunked(SX, Z, lib_elems)
        lam = w
        res = torch.zeros(m, dtype=torch.float64, device=X.device)
        for a, b in _row_chunks(n, m, lib_elems):
            res += ((SX[a:b] - X[a:b] * w) ** 2).sum(0)
        res = torch.sqrt(res)
        del SX
        worst = float(res[:r].max())
        if log:
            log(f"eigs outer {outer}: max residual {worst:.2e} ({time.time() - t0:.1f}s)")
        if worst < tol or time.time() - t0 > time_budget:
            break
        a, b = -1.0, float(w[-1])
        c, e = 0.5 * (a + b), 0.5 * (b - a)
        Y0 = X
        Y1 = (_spmm_chunked(S, X, lib_elems) - c * X) / e
        for _ in range(2, degree + 1):
            Y2 = 2.0 * (_spmm_chunked(S, Y1, lib_elems) - c * Y1) / e - Y0
            Y0, Y1 = Y1, Y2
        del Y0
        X = _orth_cholqr3(Y1, lib_elems)
        del Y1
    return (X[:, :r].cpu().numpy(), lam[:r].cpu().numpy(), res[:r].cpu().numpy())


def sparsify_eigvecs(U: np.ndarray, sparsity: float):
    """SHybrid's sparsified embeddings (Section 6.2): the smallest entries of
    U1 in magnitude are set to zero, one global threshold over the whole
    matrix, until the fraction `sparsity` of entries is zero; the kept values
    are not renormalised. Returns U1 by item in CSR form (rowptr int64[n+1],
    col int32 component ids increasing within each row, val float32)."""
    n, r = U.shape
    keep = int(round((1.0 - sparsity) * n * r))
    flat = np.abs(np.asarray(U, np.float32)).ravel()
    if keep <= 0:
        mask = np.zeros(n * r, bool)
    elif keep >= flat.size:
        mask = np.ones(n * r, bool)
    else:
        part = np.argpartition(-flat, keep - 1)[:keep]   # the keep largest magnitudes
        mask = np.zeros(n * r, bool)
        mask[part] = True
    mask = mask.reshape(n, r)
    rowptr = np.zeros(n + 1, np.int64)
    rowptr[1:] = np.cumsum(mask.sum(1))
    rows, cols = np.nonzero(mask)                       # row-major order, cols increasing
    return rowptr, cols.astype(np.int32), np.asarray(U, np.float32)[rows, cols]


def sparse_to_dense(n, r, rowptr, col, val) -> np.ndarray:
    """Dense n x r float64 copy of a CSR matrix (for the oracle)."""
    D = np.zeros((n, r))
    rows = np.repeat(np.arange(n), np.diff(rowptr))
    D[rows, col] = val
    return D


# --------------------------------------------------------------------------
# Fixture bundle
# --------------------------------------------------------------------------

@dataclass
class Fixture:
    cfg: WorkloadConfig
    V: np.ndarray            # n x d float32 database descriptors
    Q: np.ndarray            # m x d float32 queries
    rowptr: np.ndarray       # int64[n+1]
    col: np.ndarray          # int32[nnz]
    w: np.ndarray            # float64[nnz] raw weights
    s: np.ndarray            # float32[nnz] normalised values (what the GPU stores)
    U: np.ndarray            # n x r float32 eigenvectors (what the GPU stores)
    lam: np.ndarray          # r float64 eigenvalues, descending
    eig_res: np.ndarray      # r residual norms ||S u - lambda u||
    info: dict = field(default_factory=dict)

    @property
    def n(self):
        return self.cfg.n

    @property
    def nnz(self):
        return int(self.col.size)


_FIELDS = ("V", "Q", "rowptr", "col", "w", "s", "U", "lam", "eig_res")


def save_fixture(fx: Fixture, path: str) -> None:
    """Write the arrays of a fixture to a directory (one .npy per array)."""
    import json
    import os
    os.makedirs(path, exist_ok=True)
    for f in _FIELDS:
        np.save(os.path.join(path, f + ".npy"), getattr(fx, f), allow_pickle=False)
    with open(os.path.join(path, "meta.json"), "w") as fh:
        json.dump({"cfg": fx.cfg.name, "n_queries": int(fx.Q.shape[0]), "r": int(fx.U.shape[1]),
                   "info": fx.info}, fh)


def load_fixture(cfg: WorkloadConfig, path: str, n_queries: int, r: int) -> Optional[Fixture]:
    """Read a fixture written by save_fixture if it matches (cfg, n_queries, r)."""
    import json
    import os
    meta_p = os.path.join(path, "meta.json")
    if not os.path.exists(meta_p):
        return None
    meta = json.load(open(meta_p))
    if meta["cfg"] != cfg.name or meta["n_queries"] != n_queries or meta["r"] != r:
        return None
    arrs = {f: np.load(os.path.join(path, f + ".npy"), allow_pickle=False) for f in _FIELDS}
    return Fixture(cfg, info=meta["info"], **arrs)


def build_fixture(cfg: WorkloadConfig, n_queries: Optional[int] = None, r: Optional[int] = None,
                  prefer_gpu: bool = True, eig_time_budget: float = 120.0,
                  log=None, cache_dir: Optional[str] = None) -> Fixture:
    """Generate a whole workload for cfg (descriptors, queries, graph,
    eigenpairs), or read it from cache_dir when a matching copy is there."""
    nq = n_queries if n_queries is not None else cfg.batch
    rr_ = cfg.r if r is None else r
    if cache_dir:
        fx = load_fixture(cfg, cache_dir, nq, rr_)
        if fx is not None:
            return fx
    fx = _build_fixture(cfg, nq, rr_, prefer_gpu, eig_time_budget, log)
    if cache_dir:
        save_fixture(fx, cache_dir)
    return fx


def _build_fixture(cfg, n_queries, r, prefer_gpu, eig_time_budget, log) -> Fixture:
    t0 = time.time()
    say = log or (lambda *a: None)
    sc, spt, sq, se = cfg.seeds
    dev = _torch_device(prefer_gpu)
    big = dev.type == "cuda" and cfg.n >= 200_000   # generate on the GPU
    V, labels, centres = vmf_mixture(cfg.n, cfg.d, cfg.clusters, cfg.kappa, sc, spt,
                                     device=dev if big else None)
    Q = vmf_queries(n_queries, centres, cfg.kappa, sq)
    say(f"descriptors {time.time() - t0:.1f}s")
    nbr, sim = knn_lists(V, cfg.k, prefer_gpu=prefer_gpu, bf16_inputs=big)
    say(f"knn {time.time() - t0:.1f}s")
    if big:
        rowptr, col, w = mutual_knn_graph_torch(nbr, sim, cfg.n, dev)
    else:
        rowptr, col, w = mutual_knn_graph(nbr, sim, cfg.n)
    del nbr, sim
    s64 = symmetric_normalize(cfg.n, rowptr, col, w)
    s32 = s64.astype(np.float32)
    say(f"graph nnz={col.size} {time.time() - t0:.1f}s")
    rr = r
    if rr == 0:
        U = np.zeros((cfg.n, 0), np.float32)
        lam = np.zeros(0)
        res = np.zeros(0)
    elif cfg.n <= 20000:
        U64, lam, res = top_eigs_arpack(cfg.n, rowptr, col, s32.astype(np.float64), rr, se)
        U = U64.astype(np.float32)
    else:
        U64, lam, res = top_eigs_chebyshev(cfg.n, rowptr, col, s32.astype(np.float64), rr, se,
                                            time_budget=eig_time_budget, prefer_gpu=prefer_gpu, log=log)
        U = U64.astype(np.float32)
    say(f"eigs r={rr} max_res={float(res.max()) if res.size else 0:.2e} {time.time() - t0:.1f}s")
    if dev.type == "cuda":  # hand the blocks' device memory back before the library allocates
        import torch
        torch.cuda.empty_cache()
    deg = np.diff(rowptr)
    info = dict(nnz=int(col.size), mean_degree=float(deg.mean()), isolated=int((deg == 0).sum()),
                eig_max_residual=float(res.max()) if res.size else 0.0,
                build_seconds=time.time() - t0)
    return Fixture(cfg, V, Q, rowptr, col, w, s32, U, np.asarray(lam, np.float64), res, info)
