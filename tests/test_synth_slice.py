"""A q slice of a workload carries the parent's per-pair inputs (CPU)."""
import numpy as np

import synth


def test_slice_inputs_equal_parent():
    cfg = synth.make_config("ragged")
    q_ids = [4, 1]
    sl = synth.q_slice(cfg, q_ids, n_k=2)
    assert sl.n_q == 2 and sl.n_k == 2 and sl.n_bands == cfg.n_bands[:2]
    assert np.allclose(sl.weights_q(), 0.5)
    E, D, C = synth.coulomb_blocks(cfg)
    Es, Ds, Cs = synth.coulomb_blocks(sl)
    for i, q in enumerate(q_ids):
        assert sl.n_mb(i) == cfg.n_mb(q)
        assert np.array_equal(Es[i], E[q])
        for k in range(2):
            assert np.array_equal(synth.m_block(sl, k, i), synth.m_block(cfg, k, q))
    for a, b in zip(Ds + Cs, D + C):
        assert np.array_equal(a, b)
    # a slice of a slice keeps the original q numbering
    sl2 = synth.q_slice(sl, [1], n_k=1)
    assert np.array_equal(synth.m_block(sl2, 0, 0), synth.m_block(cfg, 0, 1))
