"""GPU: band pairs left out by exchange_band_mask come back as exact zeros and
the rest matches the oracle (ragged workload: 13, 37 and 21 bands, so several
8 x 8 band tiles; FP64 1e-10, bf16x3 within 4x the emulated error, both on the
kept elements with the left-out ones zero in the reference too).
"""
import functools

import numpy as np
import pytest

import synth
from oracle import chol, precision as pr, vx

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _keep(nb, seed):
    """A symmetric pair mask by 8 x 8 tiles: diagonal tiles and about half the others."""
    rng = np.random.default_rng(seed)
    nbt = (nb + 7) // 8
    tk = rng.random((nbt, nbt)) < 0.5
    tk = tk | tk.T | np.eye(nbt, dtype=bool)
    if nbt > 1:
        tk[0, -1] = tk[-1, 0] = False                        # at least one tile pair left out
    t = np.arange(nb) // 8
    return tk[t][:, t]


@pytest.mark.parametrize("precision", ["fp64", "bf16x3"])
def test_masked_tiles_are_zero_and_the_rest_matches(precision):
    import paper_1003_0524_amd as lib
    cfg = synth.make_config("ragged")
    print(f"[mask] ragged {precision}", flush=True)
    E, D, C = synth.coulomb_blocks(cfg)
    ex = lib.Exchange(cfg.n_bands, cfg.n_pw, cfg.ch_nrad, cfg.n_occ, E, D, C, w_q=cfg.weights_q(),
                      precision=precision, form="herk", batched=True)
    keeps = [_keep(nb, 30 + k) for k, nb in enumerate(cfg.n_bands)]
    for k in range(cfg.n_k):
        ex.band_mask(k, keeps[k])
    Vs = [V.cpu().numpy() for V in ex.matrix_all([torch.from_numpy(synth.m_all(cfg, k)).cuda()
                                                  for k in range(cfg.n_k)])]
    ex.band_mask(0, None)                                   # back to every pair
    V0 = ex.matrix_all([torch.from_numpy(synth.m_all(cfg, k)).cuda() for k in range(cfg.n_k)])[0].cpu().numpy()
    plan = ex.accumulation_plan()
    ex.close()
    v = [vx.assemble_v(E[q], D, C) for q in range(cfg.n_q)]
    L = [chol.cholesky(a) for a in v]
    for k in range(cfg.n_k):
        blocks = [synth.m_block(cfg, k, q) for q in range(cfg.n_q)]
        ref = np.where(keeps[k], vx.vx_k(blocks, v, cfg.weights_q()), 0)
        assert np.all(Vs[k][~keeps[k]] == 0)
        if precision == "fp64":
            assert pr.normwise_error(Vs[k], ref) <= 1e-10
        else:
            emu = np.where(keeps[k], pr.vx_k_emulated(blocks, L, cfg.weights_q(), precision, cfg.n_s, plan), 0)
            assert pr.normwise_error(Vs[k], ref) <= 4.0 * pr.normwise_error(emu, ref) + 1e-12
    assert np.any(V0[~keeps[0]] != 0)


@pytest.mark.parametrize("cid", [181, 187, 180])
def test_masked_tiles_on_the_wide_kernel(cid, monkeypatch):
    """The same on the wide kernel (complex64 M; its Gram tiles follow a per-wavefront schedule of
    band-tile units, and the mask is looked up per tile): instances 181 / 187 (bf16x3, two and one
    row tiles) and 180 (fp32)."""
    import paper_1003_0524_amd as lib
    monkeypatch.setenv("EXC_FUSED_CFG", str(cid))
    monkeypatch.delenv("EXC_FUSED", raising=False)
    precision = "fp32" if cid == 180 else "bf16x3"
    cfg = synth.make_config("ragged")
    print(f"[mask] ragged wide instance {cid}", flush=True)
    E, D, C = synth.coulomb_blocks(cfg)
    ex = lib.Exchange(cfg.n_bands, cfg.n_pw, cfg.ch_nrad, cfg.n_occ, E, D, C, w_q=cfg.weights_q(),
                      precision=precision, form="herk", batched=True)
    keeps = [_keep(nb, 40 + k) for k, nb in enumerate(cfg.n_bands)]
    for k in range(cfg.n_k):
        ex.band_mask(k, keeps[k])
    Vs = [V.cpu().numpy() for V in ex.matrix_all([torch.from_numpy(synth.m_all(cfg, k, np.complex64)).cuda()
                                                  for k in range(cfg.n_k)])]
    got = int(ex.query(3))
    plan = ex.accumulation_plan()
    ex.close()
    assert got == cid
    v = [vx.assemble_v(E[q], D, C) for q in range(cfg.n_q)]
    L = [chol.cholesky(a) for a in v]
    for k in range(cfg.n_k):
        blocks = [synth.m_block(cfg, k, q, np.complex64).astype(np.complex128) for q in range(cfg.n_q)]
        ref = np.where(keeps[k], vx.vx_k(blocks, v, cfg.weights_q()), 0)
        assert np.all(Vs[k][~keeps[k]] == 0)
        emu = np.where(keeps[k], pr.vx_k_emulated(blocks, L, cfg.weights_q(), precision, cfg.n_s, plan), 0)
        assert pr.normwise_error(Vs[k], ref) <= 4.0 * pr.normwise_error(emu, ref) + 1e-12
