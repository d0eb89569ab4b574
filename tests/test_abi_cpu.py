"""Host-only checks of the C ABI: the built library loads and exports every
entry point that include/hd.h declares, and calls that need no device fail
cleanly with a status code (no GPU is touched)."""
import ctypes
import os
import re

import pytest

from paper_1807_08692_amd import hd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "hd.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hd_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = hd.lib()
    names = declared_symbols()
    assert "hd_query_batch" in names and "hd_load_graph" in names
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(hd._SIGS), "binding and header disagree"


def test_null_context_errors_without_device():
    L = hd.lib()
    assert L.hd_load_graph(None, 1, 0, None, None, None, 0) == hd.HD_EINVAL
    assert b"NULL context" in L.hd_last_error()
    assert L.hd_load_eigs(None, 0, None, None, 0) == hd.HD_EINVAL
    assert L.hd_load_descriptors(None, 4, None, 0) == hd.HD_EINVAL
    opts = hd.hd_query_opts(0.99, 10, 1e-6, 0, 5, 10)
    assert L.hd_query_batch(None, 1, None, None, None, ctypes.byref(opts), None, None, None,
                            None, None, None, None, None, None) == hd.HD_EINVAL
    assert L.hd_rank(None, 1, 10, None, 10, 5, None, None, None) == hd.HD_EINVAL
    assert L.hd_device_bytes(None) == 0
    L.hd_destroy(None)
    out = ctypes.c_void_p()
    assert L.hd_create(-1, ctypes.byref(out)) != hd.HD_OK
    assert L.hd_create(0, None) == hd.HD_EINVAL


def test_binding_raises_on_error():
    with pytest.raises(hd.HDError):
        hd._check(hd.lib().hd_load_graph(None, 1, 0, None, None, None, 0))


def header_enum(name):
    """{enumerator: value} of a typedef enum in include/hd.h."""
    text = open(os.path.join(ROOT, "include", "hd.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    m = re.search(r"typedef enum\s*\{([^}]*)\}\s*" + name + r"\s*;", text)
    assert m, name
    return {k: int(v) for k, v in re.findall(r"(\w+)\s*=\s*(-?\d+)", m.group(1))}


def test_tuning_keys_match_header():
    """The binding's launch-parameter keys are the header's, one for one
    (hd_autotune fills HD_TUNE_NKEYS x 4 times, which the binding sizes from
    its own table)."""
    e = header_enum("hd_tune_key")
    nkeys = e.pop("HD_TUNE_NKEYS")
    assert len(hd.TUNE_KEYS) == nkeys
    assert sorted(hd.TUNE_KEYS.values()) == list(range(nkeys))
    assert sorted(e.values()) == list(range(nkeys))
    for name, k in hd.TUNE_KEYS.items():
        assert e["HD_TUNE_" + name.upper()] == k, name



def test_status_and_dtype_codes_match_header():
    """The binding's column-status and storage-type codes are the header's."""
    st = header_enum("hd_col_status")
    assert (hd.COL_CONVERGED, hd.COL_MAXITER, hd.COL_ZERO_RHS, hd.COL_BREAKDOWN) == (
        st["HD_COL_CONVERGED"], st["HD_COL_MAXITER"], st["HD_COL_ZERO_RHS"], st["HD_COL_BREAKDOWN"])
    dt = header_enum("hd_dtype")
    for name, code in hd._DTYPES.items():
        want = {"f32": "HD_F32", "bf16": "HD_BF16", "fp8": "HD_FP8_E4M3", "bf16x2": "HD_BF16X2"}[name]
        assert dt[want] == code, name
    assert dt["HD_SPARSE_F32"] == hd.HD_SPARSE_F32
    rc = header_enum("hd_status")
    assert (hd.HD_OK, hd.HD_EINVAL, hd.HD_ENOMEM, hd.HD_EDEVICE, hd.HD_ESTATE) == (
        rc["HD_OK"], rc["HD_EINVAL"], rc["HD_ENOMEM"], rc["HD_EDEVICE"], rc["HD_ESTATE"])
