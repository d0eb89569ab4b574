"""Python binding of the C ABI in include/hd.h (ctypes, argument marshalling
only). Every step of the query path runs in the library's HIP kernels;
torch supplies device buffers and streams. There is no fallback: without the
built library (``libhd.so``, see ``build.py``) every call raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhd.so")

HD_OK, HD_EINVAL, HD_ENOMEM, HD_EDEVICE, HD_ESTATE = 0, -1, -2, -3, -4
COL_CONVERGED, COL_MAXITER, COL_ZERO_RHS, COL_BREAKDOWN = 0, 1, 2, 3
HD_F32, HD_BF16, HD_FP8_E4M3, HD_BF16X2, HD_SPARSE_F32 = 0, 1, 2, 3, 4
HD_GRAPH_NORMALIZE, HD_GRAPH_CHECK_SYMMETRY = 1, 2
TOPK_MAX = 1024

_DTYPES = {"f32": HD_F32, "bf16": HD_BF16, "fp8": HD_FP8_E4M3, "bf16x2": HD_BF16X2}

# Exported entry points and their ctypes signatures (same names as hd.h).
_P = ctypes.c_void_p
_SIGS = {
    "hd_create": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_void_p)]),
    "hd_destroy": (None, [_P]),
    "hd_last_error": (ctypes.c_char_p, []),
    "hd_load_graph": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_int64, _P, _P, _P, ctypes.c_uint32]),
    "hd_load_eigs": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P, ctypes.c_int32]),
    "hd_load_descriptors": (ctypes.c_int, [_P, ctypes.c_int32, _P, ctypes.c_int32]),
    "hd_load_eigs_fp8": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P, _P]),
    "hd_load_descriptors_fp8": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P]),
    "hd_quantize_fp8_e4m3": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int32, _P, ctypes.c_int32, _P, _P]),
    "hd_load_eigs_sparse": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int64, _P, _P, _P, _P]),
    "hd_compute_eigs": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, _P, _P, _P, _P]),
    "hd_eig_steps": (ctypes.c_int32, [_P]),
    "hd_query_filter": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P, _P, ctypes.c_int32, _P, ctypes.c_int32,
                                       ctypes.c_int32, ctypes.c_int32, _P, _P, _P, _P]),
    "hd_query_batch": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P, _P, _P, _P, _P, _P, _P, _P,
                                      _P, _P, _P, _P]),
    "hd_rank": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int64, _P, ctypes.c_int64,
                               ctypes.c_int32, _P, _P, _P]),
    "hd_rank_noalloc": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int64, _P, ctypes.c_int64,
                                       ctypes.c_int32, _P, _P, _P]),
    "hd_rank_noalloc_scratch_bytes": (ctypes.c_size_t, [ctypes.c_int32, ctypes.c_int64, ctypes.c_int32]),
    "hd_probe_memory": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, _P, _P]),
    "hd_set_persistent": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int64]),
    "hd_device_bytes": (ctypes.c_int64, [_P]),
    "hd_timing_enable": (ctypes.c_int, [_P, ctypes.c_int]),
    "hd_timing_enable_kinds": (ctypes.c_int, [_P, ctypes.c_uint32]),
    "hd_timing_kinds": (ctypes.c_int, []),
    "hd_timing_name": (ctypes.c_char_p, [ctypes.c_int]),
    "hd_timing_get": (ctypes.c_int, [_P, ctypes.c_int, _P, _P]),
    "hd_serve_open": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int64, _P, ctypes.POINTER(ctypes.c_void_p)]),
    "hd_serve_column_bytes": (ctypes.c_int64, [_P, _P]),
    "hd_serve_slots": (ctypes.c_int, [_P]),
    "hd_serve_in_use": (ctypes.c_int, [_P]),
    "hd_serve_submit": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P, _P, _P, _P]),
    "hd_serve_step": (ctypes.c_int, [_P, ctypes.c_int32]),
    "hd_serve_poll": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P, _P, _P, _P, _P]),
    "hd_serve_close": (None, [_P]),
    "hd_serve_cancel": (ctypes.c_int, [_P, ctypes.c_int32, _P]),
    "hd_set_tuning": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32]),
    "hd_get_tuning": (ctypes.c_int, [_P, ctypes.c_int32, _P]),
    "hd_autotune": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, _P]),
    "hd_plan_create": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, _P, ctypes.POINTER(ctypes.c_void_p)]),
    "hd_plan_run": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "hd_plan_destroy": (None, [_P]),
    "hd_rank_plan": (ctypes.c_int, [ctypes.c_int32, _P, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_int32, _P, _P, _P, _P, _P, _P]),
}


def rank_plan(lam, cand_r, *, alpha=0.99, eps=1e-3, lambda_min=-1.0, fixed_ms=None, iter_ms=None):
    """(r, i) planner (hd_rank_plan): iterations the CG bound guarantees for
    each candidate rank, and with costs the predicted times and the best."""
    lam = np.ascontiguousarray(lam, np.float64)
    cr = np.ascontiguousarray(cand_r, np.int32)
    it = np.zeros(cr.size, np.int32)
    pm = np.zeros(cr.size, np.float64)
    best = ctypes.c_int32(-1)
    fx = np.ascontiguousarray(fixed_ms, np.float64) if fixed_ms is not None else None
    im = np.ascontiguousarray(iter_ms, np.float64) if iter_ms is not None else None
    _check(lib().hd_rank_plan(int(lam.size), lam.ctypes.data_as(_P), float(lambda_min), float(alpha),
                              float(eps), int(cr.size), cr.ctypes.data_as(_P),
                              None if fx is None else fx.ctypes.data_as(_P),
                              None if im is None else im.ctypes.data_as(_P),
                              it.ctypes.data_as(_P), pm.ctypes.data_as(_P), ctypes.byref(best)))
    return {"iters": it, "pred_ms": pm if fx is not None else None, "best": best.value}

def quantize_fp8(A, per_column: bool):
    """FP8 E4M3 quantizer of the precision form (hd_quantize_fp8_e4m3, host
    only): returns (codes uint8 rows x cols, scales fp32 per column or row)."""
    A = np.ascontiguousarray(A, np.float32)
    rows, cols = A.shape
    codes = np.zeros((rows, cols), np.uint8)
    sc = np.zeros(cols if per_column else rows, np.float32)
    _check(lib().hd_quantize_fp8_e4m3(int(rows), int(cols), A.ctypes.data_as(_P), 1 if per_column else 0,
                                      codes.ctypes.data_as(_P), sc.ctypes.data_as(_P)))
    return codes, sc


# Launch parameters (hd_tune_key)
TUNE_KEYS = {"spmm_cpl": 0, "utp_nt": 1, "uc_nt": 2, "spmm_bands": 3, "topk_onepass": 4}


class hd_eig_opts(ctypes.Structure):
    _fields_ = [("guard", ctypes.c_int32), ("degree", ctypes.c_int32), ("max_outer", ctypes.c_int32),
                ("tol", ctypes.c_double), ("time_budget_s", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("lambda_min", ctypes.c_double)]


class hd_query_opts(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("max_iter", ctypes.c_int32), ("tol", ctypes.c_double),
                ("rank_r", ctypes.c_int32), ("k_y", ctypes.c_int32), ("top_k", ctypes.c_int32)]


class HDError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (status {code})")
        self.code = code


_lib = None


def lib():
    """Load libhd.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "paper_1807_08692_amd.build.build() (hipcc, gfx950)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def last_error() -> str:
    return lib().hd_last_error().decode()


def _check(code: int):
    if code != HD_OK:
        raise HDError(code, last_error())


def _host(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data_as(ctypes.c_void_p)


def _dptr(t) -> Optional[int]:
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream) if stream.cuda_stream else None


class Context:
    """One hd_ctx on a GPU (hd_create / hd_destroy)."""

    def __init__(self, device: int = 0):
        h = ctypes.c_void_p()
        _check(lib().hd_create(int(device), ctypes.byref(h)))
        self._h = h
        self.device = device
        self.n = 0
        self.r = 0
        self.d = 0

    def close(self):
        if getattr(self, "_h", None):
            lib().hd_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ---- loaders (host arrays, copied) ----
    def load_graph(self, n, rowptr, col, val, normalize=False, check_symmetry=False):
        rp, rpp = _host(rowptr, np.int64)
        cl, clp = _host(col, np.int32)
        vl, vlp = _host(val, np.float32)
        flags = (HD_GRAPH_NORMALIZE if normalize else 0) | (HD_GRAPH_CHECK_SYMMETRY if check_symmetry else 0)
        _check(lib().hd_load_graph(self._h, int(n), int(cl.size), rpp, clp, vlp, flags))
        self.n = int(n)

    def load_eigs(self, U, lam, dtype="f32"):
        U = np.asarray(U)
        r = 0 if U.size == 0 else U.shape[1]
        Ua, Up = _host(U.reshape(self.n, r) if r else np.zeros(1, np.float32), np.float32)
        la, lp = _host(lam if r else np.zeros(1), np.float64)
        _check(lib().hd_load_eigs(self._h, r, Up, lp, _DTYPES[dtype]))
        self.r = r

    def load_eigs_fp8(self, codes, col_scale, lam):
        """U1 given as FP8 E4M3 codes (n x r uint8) and per-column scales."""
        cd, cdp = _host(codes, np.uint8)
        sc, scp = _host(col_scale, np.float32)
        la, lp = _host(lam, np.float64)
        _check(lib().hd_load_eigs_fp8(self._h, int(cd.shape[1]), cdp, scp, lp))
        self.r = int(cd.shape[1])

    def compute_eigs(self, r, dtype="f32", *, guard=None, degree=12, max_outer=60, tol=1e-9,
                     time_budget_s=0.0, seed=1, lambda_min=-1.0, want_U=False):
        """Top-r eigenpairs of the loaded S on the device (hd_compute_eigs),
        loaded into the context; returns lambda, residuals (and U if asked)."""
        o = hd_eig_opts(int(guard if guard is not None else max(20, r // 4)), int(degree), int(max_outer),
                        float(tol), float(time_budget_s), int(seed), float(lambda_min))
        lam = np.zeros(r, np.float64)
        res = np.zeros(r, np.float64)
        U = np.zeros((self.n, r), np.float32) if want_U else None
        _check(lib().hd_compute_eigs(self._h, int(r), _DTYPES[dtype], ctypes.byref(o), lam.ctypes.data_as(_P),
                                     res.ctypes.data_as(_P), None if U is None else U.ctypes.data_as(_P)))
        return {"lam": lam, "resid": res, "U": U}

    def eig_outer(self) -> int:
        """Rayleigh-Ritz steps of the last compute_eigs (hd_eig_steps)."""
        return int(lib().hd_eig_steps(self._h))

    def load_eigs_sparse(self, r, rowptr, col, val, lam):
        """Sparsified U1 (SHybrid) by item in CSR form: rowptr (n+1), col
        (component ids, increasing within a row), val (fp32); lam (r)."""
        rp_, rpp = _host(rowptr, np.int64)
        cl, clp = _host(col, np.int32)
        vl, vlp = _host(val, np.float32)
        lm, lmp = _host(lam, np.float64)
        _check(lib().hd_load_eigs_sparse(self._h, int(r), int(cl.size), rpp, clp, vlp, lmp))

    def load_descriptors(self, V, dtype="f32"):
        Va, Vp = _host(V, np.float32)
        _check(lib().hd_load_descriptors(self._h, int(Va.shape[1]), Vp, _DTYPES[dtype]))
        self.d = int(Va.shape[1])

    def load_descriptors_fp8(self, codes, row_scale):
        """Descriptors given as FP8 E4M3 codes (n x d uint8) and per-row scales."""
        cd, cdp = _host(codes, np.uint8)
        sc, scp = _host(row_scale, np.float32)
        _check(lib().hd_load_descriptors_fp8(self._h, int(cd.shape[1]), cdp, scp))
        self.d = int(cd.shape[1])

    def probe_memory(self, mode: str, bytes_: int = 1 << 30, row_bytes: int = 1024, reps: int = 5) -> dict:
        """hd_probe_memory: mode "stream", "copy", "gather" or "graph"; returns
        ms per launch, bytes per launch and GB/s."""
        ms = ctypes.c_double()
        by = ctypes.c_double()
        m = {"stream": 0, "copy": 1, "gather": 2, "graph": 3}[mode]
        _check(lib().hd_probe_memory(self._h, m, int(bytes_), int(row_bytes), int(reps), ctypes.byref(ms),
                                     ctypes.byref(by)))
        return {"ms": ms.value, "bytes": by.value, "GB_s": by.value / (ms.value * 1e-3) / 1e9}

    def set_persistent(self, mode: int, spin_limit: int = 0):
        """Persistent CG for narrow batches (hd_set_persistent): 0 off, 1 up to
        16 queries, 2 up to 64."""
        _check(lib().hd_set_persistent(self._h, int(mode), int(spin_limit)))

    def device_bytes(self) -> int:
        return int(lib().hd_device_bytes(self._h))

    def set_tuning(self, key: str, value: int):
        _check(lib().hd_set_tuning(self._h, TUNE_KEYS[key], int(value)))

    def get_tuning(self, key: str) -> int:
        v = ctypes.c_int32()
        _check(lib().hd_get_tuning(self._h, TUNE_KEYS[key], ctypes.byref(v)))
        return v.value

    def autotune(self, batch: int, reps: int = 5) -> dict:
        """Time every candidate launch parameter at this batch size and keep
        the fastest; returns {key: {value: mean ms}} and the chosen values."""
        t = (ctypes.c_double * (4 * len(TUNE_KEYS)))()
        _check(lib().hd_autotune(self._h, int(batch), int(reps), t))
        out = {}
        for name, k in TUNE_KEYS.items():
            out[name] = {"times_ms": {v: t[4 * k + j] for j, v in enumerate((1, 2, 4, 8)) if t[4 * k + j] >= 0},
                         "chosen": self.get_tuning(name)}
        return out

    def timing_enable(self, on: bool = True, kinds=None):
        """Per-kernel event timing: all kinds, or only the named ones."""
        if kinds is None or not on:
            _check(lib().hd_timing_enable(self._h, 1 if on else 0))
            return
        L = lib()
        names = {L.hd_timing_name(k).decode(): k for k in range(L.hd_timing_kinds())}
        mask = 0
        for name in kinds:
            mask |= 1 << names[name]
        _check(L.hd_timing_enable_kinds(self._h, mask))

    def timing(self) -> dict:
        """{kernel kind: (total_ms, launches)} accumulated since timing_enable."""
        L = lib()
        out = {}
        for k in range(L.hd_timing_kinds()):
            ms = ctypes.c_double()
            cnt = ctypes.c_int64()
            _check(L.hd_timing_get(self._h, k, ctypes.byref(ms), ctypes.byref(cnt)))
            out[L.hd_timing_name(k).decode()] = (ms.value, cnt.value)
        return out

    # ---- query path ----
    def query_batch(self, q_desc=None, y_ids=None, y_val=None, *, alpha=0.99, max_iter=20,
                    tol=1e-6, rank_r=-1, k_y=10, top_k=100, want_x=False, want_y=False,
                    stream=None, out=None):
        """Run the whole query path on B queries. q_desc: torch (B x d fp32,
        device) or None with y_ids / y_val (B x k_y int32 / fp32, device).
        Returns a dict of device tensors (rank_ids, rank_scores, x, y_ids,
        y_val) and host arrays (iters, relres, status)."""
        import torch
        dev = torch.device("cuda", self.device)
        if q_desc is not None:
            B = int(q_desc.shape[0])
        else:
            B = int(y_ids.shape[0])
            k_y = int(y_ids.shape[1])
        o = hd_query_opts(float(alpha), int(max_iter), float(tol), int(rank_r), int(k_y), int(top_k))
        res = out if out is not None else {}
        if top_k > 0:
            res.setdefault("rank_ids", torch.empty((B, top_k), dtype=torch.int32, device=dev))
            res.setdefault("rank_scores", torch.empty((B, top_k), dtype=torch.float32, device=dev))
        if want_x:
            res.setdefault("x", torch.empty((B, self.n), dtype=torch.float32, device=dev))
        if want_y:
            res.setdefault("y_ids", torch.empty((B, k_y), dtype=torch.int32, device=dev))
            res.setdefault("y_val", torch.empty((B, k_y), dtype=torch.float32, device=dev))
        it = res.setdefault("iters", np.zeros(B, np.int32))
        rr = res.setdefault("relres", np.zeros(B, np.float64))
        st = res.setdefault("status", np.zeros(B, np.int32))
        code = lib().hd_query_batch(
            self._h, B, _dptr(q_desc), _dptr(y_ids), _dptr(y_val), ctypes.byref(o),
            _dptr(res.get("rank_ids")), _dptr(res.get("rank_scores")), _dptr(res.get("x")),
            _dptr(res.get("y_ids")), _dptr(res.get("y_val")),
            it.ctypes.data_as(_P), rr.ctypes.data_as(_P), st.ctypes.data_as(_P),
            _stream_ptr(stream))
        _check(code)
        return res

    def query_filter(self, coeffs, q_desc=None, y_ids=None, y_val=None, *, rank_r=-1, k_y=10, top_k=100,
                     want_x=False, stream=None):
        """Polynomial filter h(S) y, h(x) = sum_i coeffs[i] x^i (hd_query_filter)."""
        import torch
        dev = torch.device("cuda", self.device)
        if q_desc is not None:
            B = int(q_desc.shape[0])
        else:
            B = int(y_ids.shape[0])
            k_y = int(y_ids.shape[1])
        c, cp = _host(coeffs, np.float64)
        res = {}
        if top_k > 0:
            res["rank_ids"] = torch.empty((B, top_k), dtype=torch.int32, device=dev)
            res["rank_scores"] = torch.empty((B, top_k), dtype=torch.float32, device=dev)
        if want_x:
            res["x"] = torch.empty((B, self.n), dtype=torch.float32, device=dev)
        _check(lib().hd_query_filter(self._h, B, _dptr(q_desc), _dptr(y_ids), _dptr(y_val), int(c.size) - 1, cp,
                                     int(rank_r), int(k_y), int(top_k), _dptr(res.get("rank_ids")),
                                     _dptr(res.get("rank_scores")), _dptr(res.get("x")), _stream_ptr(stream)))
        return res

    def rank(self, x, K, stream=None, ids=None, scores=None):
        """Top-K of each row of x (torch, B x n fp32, device)."""
        import torch
        B, n = int(x.shape[0]), int(x.shape[1])
        ldx = int(x.stride(0))
        if ids is None:
            ids = torch.empty((B, K), dtype=torch.int32, device=x.device)
        if scores is None:
            scores = torch.empty((B, K), dtype=torch.float32, device=x.device)
        _check(lib().hd_rank(self._h, B, n, _dptr(x), ldx, int(K), _dptr(ids), _dptr(scores),
                             _stream_ptr(stream)))
        return ids, scores


    def rank_noalloc(self, x, K, stream=None, ids=None, scores=None):
        """hd_rank_noalloc: the top-K of each row of x with the library's fixed
        scratch (no device allocation in the call)."""
        import torch
        B, n = int(x.shape[0]), int(x.shape[1])
        if ids is None:
            ids = torch.empty((B, K), dtype=torch.int32, device=x.device)
        if scores is None:
            scores = torch.empty((B, K), dtype=torch.float32, device=x.device)
        _check(lib().hd_rank_noalloc(self._h, B, n, _dptr(x), int(x.stride(0)), int(K), _dptr(ids), _dptr(scores),
                                     _stream_ptr(stream)))
        return ids, scores


class Plan:
    """A query plan: the whole query path for B queries captured into a HIP
    graph (hd_plan_*). input: "descriptors" or "y"."""

    def __init__(self, ctx: "Context", B: int, input: str = "descriptors", *, alpha=0.99, max_iter=20,
                 tol=1e-6, rank_r=-1, k_y=10, top_k=100):
        self.ctx, self.B, self.top_k, self.k_y = ctx, int(B), int(top_k), int(k_y)
        self.input = {"descriptors": 0, "y": 1}[input]
        o = hd_query_opts(float(alpha), int(max_iter), float(tol), int(rank_r), int(k_y), int(top_k))
        h = ctypes.c_void_p()
        _check(lib().hd_plan_create(ctx._h, self.B, self.input, ctypes.byref(o), ctypes.byref(h)))
        self._h = h

    def run(self, q_desc=None, y_ids=None, y_val=None, stream=None, out=None) -> dict:
        """Run on device tensors (q_desc B x d, or y_ids / y_val B x k_y);
        returns rank_ids / rank_scores (device) and iters / relres / status."""
        import torch
        dev = torch.device("cuda", self.ctx.device)
        res = out if out is not None else {}
        res.setdefault("rank_ids", torch.empty((self.B, self.top_k), dtype=torch.int32, device=dev))
        res.setdefault("rank_scores", torch.empty((self.B, self.top_k), dtype=torch.float32, device=dev))
        it = res.setdefault("iters", np.zeros(self.B, np.int32))
        rr = res.setdefault("relres", np.zeros(self.B, np.float64))
        st = res.setdefault("status", np.zeros(self.B, np.int32))
        _check(lib().hd_plan_run(self._h, _dptr(q_desc), _dptr(y_ids), _dptr(y_val),
                                 _dptr(res["rank_ids"]), _dptr(res["rank_scores"]),
                                 it.ctypes.data_as(_P), rr.ctypes.data_as(_P), st.ctypes.data_as(_P),
                                 _stream_ptr(stream)))
        return res

    def close(self):
        if getattr(self, "_h", None):
            lib().hd_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching server on a context (hd_serve_*). Requests are
    host arrays; results come back as host arrays."""

    def __init__(self, ctx: Context, slots: int, *, hbm_budget_bytes: int = 0, alpha=0.99,
                 max_iter=20, tol=1e-6, rank_r=-1, k_y=10, top_k=100):
        o = hd_query_opts(float(alpha), int(max_iter), float(tol), int(rank_r), int(k_y), int(top_k))
        h = ctypes.c_void_p()
        _check(lib().hd_serve_open(ctx._h, int(slots), int(hbm_budget_bytes), ctypes.byref(o),
                                   ctypes.byref(h)))
        self._h = h
        self.ctx = ctx  # keeps the context alive
        self.k_y = int(k_y)
        self.top_k = int(top_k)
        self.tol = float(tol)

    @staticmethod
    def column_bytes(ctx: Context, *, alpha=0.99, max_iter=20, tol=1e-6, rank_r=-1, k_y=10, top_k=100) -> int:
        o = hd_query_opts(float(alpha), int(max_iter), float(tol), int(rank_r), int(k_y), int(top_k))
        return int(lib().hd_serve_column_bytes(ctx._h, ctypes.byref(o)))

    @property
    def slots(self) -> int:
        return int(lib().hd_serve_slots(self._h))

    @property
    def in_use(self) -> int:
        return int(lib().hd_serve_in_use(self._h))

    def submit(self, y_ids=None, y_val=None, q_desc=None, max_iter=None):
        """Admit requests into free columns; returns the tickets of the
        admitted prefix (length = number admitted)."""
        if q_desc is not None:
            q, qp = _host(q_desc, np.float32)
            n = q.shape[0]
            ip = vp = None
        else:
            yi, ip = _host(y_ids, np.int32)
            yv, vp = _host(y_val, np.float32)
            n = yi.shape[0]
            qp = None
        mp = None
        if max_iter is not None:
            mi, mp = _host(np.broadcast_to(np.asarray(max_iter, np.int32), (n,)), np.int32)
        tickets = np.zeros(max(n, 1), np.int64)
        got = lib().hd_serve_submit(self._h, n, qp, ip, vp, mp, tickets.ctypes.data_as(_P))
        if got < 0:
            _check(got)
        return tickets[:got]

    def step(self, iters: int = 1):
        _check(lib().hd_serve_step(self._h, int(iters)))

    def cancel(self, tickets) -> int:
        """Cancel admitted, uncollected requests; returns how many were."""
        t, tp = _host(np.atleast_1d(np.asarray(tickets, np.int64)), np.int64)
        got = lib().hd_serve_cancel(self._h, int(t.size), tp)
        if got < 0:
            _check(got)
        return got

    def poll(self, max_out: int = 1024):
        """Finished requests: dict of arrays keyed tickets, ids, scores,
        iters, relres, status (ids / scores: n x top_k)."""
        t = np.zeros(max_out, np.int64)
        ids = np.zeros((max_out, self.top_k), np.int32)
        sc = np.zeros((max_out, self.top_k), np.float32)
        it = np.zeros(max_out, np.int32)
        rr = np.zeros(max_out, np.float64)
        st = np.zeros(max_out, np.int32)
        got = lib().hd_serve_poll(self._h, int(max_out), t.ctypes.data_as(_P), ids.ctypes.data_as(_P),
                                  sc.ctypes.data_as(_P), it.ctypes.data_as(_P), rr.ctypes.data_as(_P),
                                  st.ctypes.data_as(_P))
        if got < 0:
            _check(got)
        return dict(tickets=t[:got], ids=ids[:got], scores=sc[:got], iters=it[:got], relres=rr[:got],
                    status=st[:got])

    def close(self):
        if getattr(self, "_h", None):
            lib().hd_serve_close(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
