"""The inversion-symmetric (real) variant, checked on the CPU with the oracle.

With real v(q) (inversion symmetry, Sec. III.D) and real projections, the exchange
matrix is real symmetric. The library computes it from bands packed in pairs as
complex columns (column j = M_{2j} + i M_{2j+1}); since v is real,
Re(A^H v A) of a packed column is the sum of the two bands' A^T v A. This file
checks that identity, and the layout of the packing helper, with the oracle.
"""
import numpy as np
import pytest

import synth
from oracle import vx


@pytest.mark.parametrize("name", ["tiny", "small", "ragged"])
def test_packed_pairs_give_the_real_exchange_matrix(name):
    cfg = synth.make_config(name)
    E, D, C = synth.coulomb_blocks_real(cfg)
    v = [vx.assemble_v(E[q], D, C) for q in range(cfg.n_q)]
    for q in range(cfg.n_q):
        assert np.all(v[q].imag == 0) and np.linalg.eigvalsh(v[q].real).min() > 0
    for k in range(cfg.n_k):
        mr = [synth.m_block_real(cfg, k, q) for q in range(cfg.n_q)]
        ref = vx.vx_k(mr, v, cfg.weights_q())
        assert np.all(ref.imag == 0)                                 # real inputs, real result
        assert np.allclose(ref, ref.T, rtol=0, atol=1e-12 * np.abs(ref).max())
        assert np.linalg.eigvalsh(ref.real).max() <= 1e-12 * np.abs(ref).max()   # v PD => V NSD
        packed = vx.vx_k([synth.pack_real_pairs(m) for m in mr], v, cfg.weights_q())
        assert np.max(np.abs(packed.real - ref.real)) <= 1e-13 * np.abs(ref).max()


def test_pack_real_pairs_layout():
    m = np.arange(5 * 2 * 3, dtype=np.float64).reshape(5, 2, 3)
    p = synth.pack_real_pairs(m)
    assert p.shape == (3, 2, 3) and p.dtype == np.complex128
    assert np.array_equal(p[1].real, m[2]) and np.array_equal(p[1].imag, m[3])
    assert np.array_equal(p[2].real, m[4]) and not np.any(p[2].imag)
    flat = synth.m_all_real_packed(synth.make_config("small"), 0)
    cfg = synth.make_config("small")
    assert flat.size == sum((cfg.n_occ + 1) // 2 * cfg.n_bands[0] * cfg.n_mb(q) for q in range(cfg.n_q))
