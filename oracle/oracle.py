"""FP64 oracle for hybrid spectral-temporal diffusion.

TEST INFRASTRUCTURE ONLY. This module wraps the plain C oracle in
``hd_oracle.c`` and adds the few dense references that are simplest as a
library call (a Cholesky solve, a symmetric eigen-decomposition). Only the
test suite, the smoke check and the CPU-baseline leg of the benchmark may
import it; the GPU library never does, and it imports nothing from the GPU
library.

Every function works in float64. Single-precision inputs (the graph values,
descriptors and eigenvectors the GPU also receives) are widened exactly.

Entry points and the passage each follows (Iscen et al., "Hybrid Diffusion:
Spectral-Temporal Graph Filtering for Manifold Ranking"):

* ``normalize``      Section 3: S = D^-1/2 W D^-1/2.
* ``observation``    Sections 3 and 6.1: top-k neighbours, entries (v^T z)_+^3.
* ``spectral``       Section 4.2, eq. (h-spectral).
* ``cg``             Section 4.2, eqs. (h-temporal) and (box); Section 5.
* ``iterate``        eq. (hybrid): spectral term plus the CG temporal term,
                     the exact FP64 counterpart of the GPU path.
* ``truth_dense``    Section 3, eqs. (temporal) and (transfer):
                     x* = (1 - alpha)(I - alpha S)^-1 y by Cholesky.
* ``method_dense``   eq. (hybrid) with the temporal system of eq. (h-temporal)
                     solved exactly (dense), for tiny graphs.
* ``rank``           Section 3: decreasing x, ties to the lower id.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hd_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libhd_oracle.so")

CONVERGED, MAXITER, ZERO_RHS, BREAKDOWN = 0, 1, 2, 3


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (no fast-math: IEEE double semantics)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared",
                               "-fno-fast-math", "-ffp-contract=off",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        i64, i32, f64 = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        L.hdo_normalize.argtypes = [i64, P, P, P, P]
        L.hdo_normalize.restype = ctypes.c_int
        L.hdo_csr_matvec.argtypes = [i64, P, P, P, P, P]
        L.hdo_csr_matvec.restype = None
        L.hdo_observation.argtypes = [i64, i64, P, P, i32, P, P]
        L.hdo_observation.restype = ctypes.c_int
        L.hdo_spectral.argtypes = [i64, i32, P, P, f64, i32, P, P, P]
        L.hdo_spectral.restype = ctypes.c_int
        L.hdo_cg.argtypes = [i64, P, P, P, i32, P, P, f64, P, i32, f64, P, P, P, P]
        L.hdo_cg.restype = ctypes.c_int
        L.hdo_rank.argtypes = [i64, P, i32, P, P]
        L.hdo_rank.restype = ctypes.c_int
        _lib = L
    return _lib


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class Graph64:
    """CSR graph widened to float64 / int64 row pointers for the oracle."""
    n: int
    rowptr: np.ndarray
    col: np.ndarray
    val: np.ndarray

    @staticmethod
    def from_csr(n, rowptr, col, val) -> "Graph64":
        return Graph64(int(n), _c(rowptr, np.int64), _c(col, np.int32), _c(val, np.float64))

    def dense(self) -> np.ndarray:
        A = np.zeros((self.n, self.n))
        for i in range(self.n):
            s, e = self.rowptr[i], self.rowptr[i + 1]
            A[i, self.col[s:e]] = self.val[s:e]
        return A


def normalize(n, rowptr, col, w) -> np.ndarray:
    """Section 3: values of D^-1/2 W D^-1/2 on W's sparsity pattern."""
    rp, cl, wv = _c(rowptr, np.int64), _c(col, np.int32), _c(w, np.float64)
    out = np.empty_like(wv)
    if lib().hdo_normalize(int(n), _p(rp), _p(cl), _p(wv), _p(out)) != 0:
        raise MemoryError("hdo_normalize")
    return out


def csr_matvec(g: Graph64, z) -> np.ndarray:
    z = _c(z, np.float64)
    out = np.empty(g.n)
    lib().hdo_csr_matvec(g.n, _p(g.rowptr), _p(g.col), _p(g.val), _p(z), _p(out))
    return out


def observation(V, q, k):
    """Sections 3 and 6.1: (ids, values) of one query's sparse y, best first."""
    V, q = _c(V, np.float64), _c(q, np.float64)
    n, d = V.shape
    ids = np.empty(k, np.int32)
    vals = np.empty(k, np.float64)
    if lib().hdo_observation(n, d, _p(V), _p(q), int(k), _p(ids), _p(vals)) != 0:
        raise ValueError("hdo_observation: bad k")
    return ids, vals


def similarities(V, q) -> np.ndarray:
    """All n cosines q^T v_j in FP64 (used to judge near-ties of top-k sets)."""
    return _c(V, np.float64) @ _c(q, np.float64)


def spectral(U, lam, alpha, y_ids, y_val, n=None) -> np.ndarray:
    """Section 4.2, eq. (h-spectral): x^s = U1 g(L1) U1^T y for sparse y."""
    U = _c(U, np.float64)
    if U.ndim != 2:
        raise ValueError("U must be n x r")
    n_, r = U.shape
    n = n_ if n is None else n
    lam = _c(lam, np.float64)
    ids, val = _c(y_ids, np.int32), _c(y_val, np.float64)
    out = np.empty(n)
    if r == 0:
        out[:] = 0.0
        return out
    if lib().hdo_spectral(n, r, _p(U), _p(lam), float(alpha), len(ids), _p(ids), _p(val), _p(out)) != 0:
        raise MemoryError("hdo_spectral")
    return out


def cg(g: Graph64, U, lam, alpha, y, max_iter, tol):
    """Section 4.2, eqs. (h-temporal), (box); Section 5. Returns
    (x, iters, relres, status)."""
    if U is None:
        U = np.zeros((g.n, 0))
        lam = np.zeros(0)
    U = _c(U, np.float64)
    r = U.shape[1] if U.size else 0
    lam = _c(lam, np.float64)
    y = _c(y, np.float64)
    x = np.empty(g.n)
    it = ctypes.c_int32()
    rr = ctypes.c_double()
    st = ctypes.c_int32()
    Up = _p(U) if r else None
    lp = _p(lam) if r else None
    if lib().hdo_cg(g.n, _p(g.rowptr), _p(g.col), _p(g.val), r, Up, lp, float(alpha),
                    _p(y), int(max_iter), float(tol), _p(x),
                    ctypes.byref(it), ctypes.byref(rr), ctypes.byref(st)) != 0:
        raise MemoryError("hdo_cg")
    return x, it.value, rr.value, st.value


def dense_y(n, ids, vals) -> np.ndarray:
    y = np.zeros(n)
    np.add.at(y, np.asarray(ids, np.int64), np.asarray(vals, np.float64))
    return y


def iterate(g: Graph64, U, lam, alpha, y_ids, y_val, max_iter, tol):
    """eq. (hybrid): x = x^s + x^t with x^t from CG (the GPU algorithm in
    FP64). Returns (x, x_s, x_t, iters, relres, status)."""
    r = 0 if U is None else np.asarray(U).shape[1]
    xs = spectral(U, lam, alpha, y_ids, y_val, n=g.n) if r else np.zeros(g.n)
    xt, it, rr, st = cg(g, U, lam, alpha, dense_y(g.n, y_ids, y_val), max_iter, tol)
    return xs + xt, xs, xt, it, rr, st


def filter_poly(g: Graph64, U, lam, coeffs, y_ids, y_val) -> np.ndarray:
    """Appendix A, eqs. (series), (2-main), (2-aux): for a polynomial
    h(x) = sum_i c_i x^i, x = h(S) y = U1 g(L1) U1^T y + h(S_r) y with
    g(x) = h(x) - h(0) and S_r = S - U1 L1 U1^T. The temporal term is the sum
    of c_i S_r^i y written out term by term (powers of S_r applied in turn);
    double precision throughout."""
    c = _c(coeffs, np.float64)
    y = dense_y(g.n, y_ids, y_val)
    r = 0 if U is None else np.asarray(U).shape[1]
    x = np.zeros(g.n)
    if r:
        U = _c(U, np.float64)
        lam = _c(lam, np.float64)
        gl = np.zeros(r)
        for i in range(1, c.size):
            gl += c[i] * lam ** i
        x += U @ (gl * (U.T @ y))
    v = y.copy()
    x += c[0] * v
    for i in range(1, c.size):
        v = csr_matvec(g, v) - (U @ (lam * (U.T @ v)) if r else 0.0)
        x += c[i] * v
    return x


def truth_dense(S_dense: np.ndarray, alpha, y) -> np.ndarray:
    """Section 3, eqs. (temporal), (transfer): x* = (1 - alpha)(I - alpha S)^-1 y.
    I - alpha S is symmetric positive definite (spectrum of S in [-1, 1] and
    alpha < 1), so a Cholesky factorisation (library primitive) solves it."""
    import scipy.linalg as sla
    n = S_dense.shape[0]
    A = np.eye(n) - alpha * S_dense
    c = sla.cho_factor(A, lower=True)
    return (1.0 - alpha) * sla.cho_solve(c, np.asarray(y, np.float64))


def method_dense(S_dense: np.ndarray, U, lam, alpha, y) -> np.ndarray:
    """eq. (hybrid) with both terms exact: x^s by eq. (h-spectral) and x^t by a
    dense solve of eq. (h-temporal), L(S - U1 L1 U1^T) x^t = y."""
    import scipy.linalg as sla
    n = S_dense.shape[0]
    y = np.asarray(y, np.float64)
    U = np.asarray(U, np.float64).reshape(n, -1)
    lam = np.asarray(lam, np.float64)
    g = (1.0 - alpha) / (1.0 - alpha * lam) - (1.0 - alpha)
    xs = U @ (g * (U.T @ y))
    Sr = S_dense - (U * lam) @ U.T
    L = (np.eye(n) - alpha * Sr) / (1.0 - alpha)
    xt = sla.solve(L, y, assume_a="sym")
    return xs + xt


def rank(x, K):
    """Section 3: top-K (ids, scores) by decreasing x, ties to the lower id."""
    x = _c(x, np.float64)
    n = x.shape[0]
    ids = np.empty(K, np.int32)
    sc = np.empty(K, np.float64)
    if lib().hdo_rank(n, _p(x), int(K), _p(ids), _p(sc)) != 0:
        raise ValueError("hdo_rank: bad K")
    return ids, sc


def query(g: Graph64, U, lam, alpha, V, q, k_y, max_iter, tol, K):
    """The whole query path in FP64: y, x^s, x^t, ranking of x."""
    ids, vals = observation(V, q, k_y)
    x, xs, xt, it, rr, st = iterate(g, U, lam, alpha, ids, vals, max_iter, tol)
    rid, rsc = rank(x, K)
    return dict(y_ids=ids, y_val=vals, x=x, xs=xs, xt=xt, iters=it, relres=rr,
                status=st, rank_ids=rid, rank_scores=rsc)
