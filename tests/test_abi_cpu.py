"""The C-ABI library loads and exports every symbol include/exchange.h declares.

No compute calls: these run without a GPU. Only argument validation that the
library performs before touching the device is exercised.
"""
import ctypes
import os
import re

import pytest

import paper_1003_0524_amd as pkg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "exchange.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(exchange_[a-z_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(pkg.LIB_PATH):
        pytest.fail("libexchange.so is not built (run python -m paper_1003_0524_amd.build)")
    return pkg.load_library()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert set(names) == set(pkg.EXPORTED_SYMBOLS)
    for n in names:
        assert hasattr(lib, n), n


def test_init_rejects_null_arguments_without_gpu(lib):
    out = ctypes.c_void_p(123)
    st = lib.exchange_init(None, None, None, ctypes.byref(out))
    assert st == -1 and out.value is None
    assert b"NULL" in lib.exchange_last_error(None)
    assert lib.exchange_init(None, None, None, None) == -1


def test_init_rejects_bad_sizes_without_gpu(lib):
    nb = (ctypes.c_int32 * 1)(4)
    pw = (ctypes.c_int32 * 1)(3)
    ch = (ctypes.c_int32 * 1)(0)          # nrad < 1 is invalid
    d = pkg._Desc(1, 1, 1, 1, nb, pw, ch, None, 0, 1, 1, 0)
    e = (ctypes.c_void_p * 1)(None)
    c = pkg._Coulomb(e, None, None, 0)
    out = ctypes.c_void_p()
    assert lib.exchange_init(ctypes.byref(d), ctypes.byref(c), None, ctypes.byref(out)) == -1
    d = pkg._Desc(0, 1, 1, 0, nb, pw, None, None, 0, 1, 1, 0)
    assert lib.exchange_init(ctypes.byref(d), ctypes.byref(c), None, ctypes.byref(out)) == -1
    d = pkg._Desc(1, 1, 1, 0, nb, pw, None, None, 7, 1, 1, 0)     # bad precision
    assert lib.exchange_init(ctypes.byref(d), ctypes.byref(c), None, ctypes.byref(out)) == -1
    d = pkg._Desc(1, 1, 1, 0, nb, pw, None, None, 2, 0, 1, 0)     # GEMM form is FP64 only
    assert lib.exchange_init(ctypes.byref(d), ctypes.byref(c), None, ctypes.byref(out)) == -6
    pw0 = (ctypes.c_int32 * 1)(0)
    d = pkg._Desc(1, 1, 1, 0, nb, pw0, None, None, 0, 1, 1, 0)    # empty mixed basis
    assert lib.exchange_init(ctypes.byref(d), ctypes.byref(c), None, ctypes.byref(out)) == -1
    assert b"empty" in lib.exchange_last_error(None)
    nb_big = (ctypes.c_int32 * 1)(129)
    d = pkg._Desc(1, 1, 1, 0, nb_big, pw, None, None, 0, 1, 1, 0)
    assert lib.exchange_init(ctypes.byref(d), ctypes.byref(c), None, ctypes.byref(out)) == -6


def test_null_context_calls(lib):
    v = ctypes.c_double()
    assert lib.exchange_query(None, 0, ctypes.byref(v)) == -1
    assert lib.exchange_matrix(None, 0, None, 0, 1, None, None) == -1
    assert lib.exchange_matrix_noalloc(None, 0, None, 0, None, None) == -1
    assert lib.exchange_matrix_all(None, None, 0, 1, None, None) == -1
    assert lib.exchange_energy(None, None, None, ctypes.byref(v)) == -1
    assert lib.exchange_gamma_term(None, None, None, 0.005, 1, ctypes.byref(v), None) == -1
    assert lib.exchange_back_transform(None, 0, None, 1, None, None) == -1
    assert lib.exchange_band_mask(None, 0, None) == -1
    lib.exchange_destroy(None)


def test_binding_fails_loudly_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    with pytest.raises(pkg.ExchangeError):
        pkg.Exchange([4], [3], [2], 1, [None], [None], [None])
