"""The C ABI without a GPU: the library loads, exports every symbol the header
declares, and rejects bad arguments before touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1901_09266_amd as dode
from paper_1901_09266_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "dode.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^(?:const\s+)?\w+\*?\s+\**(\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1901_09266_amd.build import build
        build()
    return _lib.lib()


def test_exports_every_declared_symbol(L):
    names = header_functions()
    assert len(names) >= 12
    assert sorted(names) == sorted(_lib.EXPORTS)
    for n in names:
        assert hasattr(L, n), n


def test_defaults(L):
    p = dode.spgd_defaults()
    assert (p.epochs, p.batch_rows, p.eta, p.eps, p.optimizer) == (300, 8192, 5.0, 1e-10, 0)


def _create(L, dims, rp, ci, vals, storage=1):
    ptrs = (ctypes.POINTER(ctypes.c_double) * len(vals))(
        *[v.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) for v in vals])
    out = ctypes.c_void_p()
    st = L.dar_create(ctypes.byref(_lib.Dims(*dims)), len(vals),
                      rp.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                      ci.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), ptrs, storage,
                      ctypes.c_void_p(0), ctypes.byref(out))
    return st, out


def test_dar_create_rejects_bad_input(L):
    P, Ld, T, H, K = 3, 2, 4, 4, 2
    rp = np.array([0, 2, 3], dtype=np.int32)
    ci = np.array([0, 2, 1], dtype=np.int32)
    good = np.ones((K, T, 3))
    st, _ = _create(L, (P, Ld, T, H, 0), rp, ci, [good])
    assert st == _lib.DODE_ERR_SHAPE and b"dims" in L.dode_last_error()
    st, _ = _create(L, (P, Ld, T, H, K), np.array([1, 2, 3], dtype=np.int32), ci, [good])
    assert st == _lib.DODE_ERR_SHAPE
    st, _ = _create(L, (P, Ld, T, H, K), rp, np.array([0, 3, 1], dtype=np.int32), [good])
    assert st == _lib.DODE_ERR_SHAPE and b"col_idx" in L.dode_last_error()
    st, _ = _create(L, (P, Ld, T, H, K), rp, np.array([2, 0, 1], dtype=np.int32), [good])
    assert st == _lib.DODE_ERR_SHAPE
    st, _ = _create(L, (P, Ld, T, H, K), rp, ci, [good], storage=9)
    assert st == _lib.DODE_ERR_DTYPE
    bad = good.copy()
    bad[1, 0, 2] = np.nan
    st, _ = _create(L, (P, Ld, T, H, K), rp, ci, [bad])
    assert st == _lib.DODE_ERR_NONFINITE
    # a NaN in a block past the last interval is ignored by definition, so only
    # in-range blocks are scanned: t + l >= H entries are never read
    st, _ = _create(L, (P, Ld, T, H, 70), rp, ci, [np.ones((70, T, 3))])
    assert st == _lib.DODE_ERR_SHAPE


def test_null_handles_and_params(L):
    assert L.dode_loss(None, 0, None, None, 1, None, None) == _lib.DODE_ERR_ARG
    assert b"NULL" in L.dode_last_error()
    assert L.dode_apply(None, 0, None, 1, None, None) == _lib.DODE_ERR_ARG
    assert L.dode_grad(None, 0, None, None, 1, None, None) == _lib.DODE_ERR_ARG
    assert L.dode_metrics(None, 0, None, None, 1, None, None, None, None) == _lib.DODE_ERR_ARG
    assert L.dar_set_values(None, 0, None, None) == _lib.DODE_ERR_ARG
    assert L.dar_destroy(None) == _lib.DODE_OK
    p = _lib.make_params(epochs=-1)
    dc = np.zeros(1, dtype=np.int32)
    assert L.spgd_solve(None, dc.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), 1, None, None, None,
                        ctypes.byref(p), None, 0, None, None) == _lib.DODE_ERR_ARG


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        _lib.lib()
