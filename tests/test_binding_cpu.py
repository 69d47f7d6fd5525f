"""The Python binding refuses a mis-sized M or output before any launch (CPU only).

The kernels size their reads from the context's shapes, so a short M, or one that
still holds the q blocks of pairs a per-pair weight of zero leaves out, must be
refused by the binding. The binding object is set up here without a context (no GPU
needed): the checks run before the C library is called.
"""
import numpy as np
import pytest
import torch

import paper_1003_0524_amd as pkg


def _fake(n_bands, n_pw, ch_nrad, n_occ, w_kq=None):
    ex = pkg.Exchange.__new__(pkg.Exchange)
    ex._torch = torch
    ex.n_k, ex.n_q = len(n_bands), len(n_pw)
    ex.n_bands = list(n_bands)
    ex.n_occ = n_occ
    ex.n_cols = n_occ
    ex.inversion = False
    ex.pair_used = np.ones((ex.n_k, ex.n_q), bool) if w_kq is None else np.asarray(w_kq) != 0
    n_s = sum(b - 1 for b in ch_nrad)
    ex.n_mb = [n_s + len(ch_nrad) + p for p in n_pw]
    ex.ctx = None
    return ex


def test_short_m_is_refused():
    ex = _fake([4, 6], [5, 7, 3], [3, 1, 2], 2)
    want = ex.m_elems(1)
    assert want == 2 * 6 * sum(ex.n_mb)
    with pytest.raises(pkg.ExchangeError) as e:
        ex.matrix(1, torch.zeros(want - 1, dtype=torch.complex128))
    assert e.value.status == -1 and "elements" in str(e.value)
    with pytest.raises(pkg.ExchangeError):
        ex.matrix_host(1, np.zeros(want - 1, np.complex128))
    with pytest.raises(pkg.ExchangeError):
        ex.matrix_all([torch.zeros(ex.m_elems(0), dtype=torch.complex64),
                       torch.zeros(want + 3, dtype=torch.complex64)])


def test_m_with_left_out_blocks_is_refused():
    w = np.array([[0.5, 0.0, 0.5], [0.0, 1.0, 0.0]])
    ex = _fake([4, 6], [5, 7, 3], [3, 1, 2], 2, w_kq=w)
    full = 2 * 4 * sum(ex.n_mb)
    kept = 2 * 4 * (ex.n_mb[0] + ex.n_mb[2])
    assert ex.m_elems(0) == kept
    with pytest.raises(pkg.ExchangeError) as e:
        ex.matrix(0, torch.zeros(full, dtype=torch.complex128))   # still holds the q = 1 block
    assert e.value.status == -1


def test_bad_output_is_refused():
    ex = _fake([4], [5], [2], 1)
    M = torch.zeros(ex.m_elems(0), dtype=torch.complex128)
    with pytest.raises(pkg.ExchangeError):
        ex.matrix(0, M, out=torch.zeros(15, dtype=torch.complex128))
    with pytest.raises(pkg.ExchangeError):
        ex.matrix(0, M, out=torch.zeros(16, dtype=torch.complex64))
    with pytest.raises(pkg.ExchangeError):
        ex.matrix(0, torch.zeros(ex.m_elems(0), dtype=torch.float64))
