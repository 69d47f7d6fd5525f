"""GPU parity on degenerate shapes: no muffin-tin channels (plane waves only), q points
without plane waves (muffin-tin only), channels without multipole-free functions, and a
single band with a single occupied band, and the largest band count (128). Same bars as
the parity tests.
"""
import math

import numpy as np
import pytest

import synth
from oracle import chol, precision as pr, vx

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _cfg(name):
    rng = np.random.default_rng([17, len(name)])
    q = rng.uniform(0.0, 1.0, size=(3, 3))
    sc = 8.0 * np.eye(3)
    if name == "pw_only":
        return synth.Config(name, 21, 0, sc, q, n_k=2, n_occ=2, n_bands=[5, 9], ch_nrad=[], n_pw=[20, 31, 12])
    if name == "mt_only_q":
        return synth.Config(name, 22, 0, sc, q, n_k=2, n_occ=1, n_bands=[1, 3], ch_nrad=[3, 1, 4, 2],
                            n_pw=[0, 7, 0])
    if name == "max_bands":                       # the largest band count the library takes
        return synth.Config(name, 24, 0, sc, q, n_k=1, n_occ=3, n_bands=[128], ch_nrad=[3, 2, 5],
                            n_pw=[40, 21, 33])
    if name == "one_band":
        return synth.Config(name, 23, 0, sc, q, n_k=1, n_occ=1, n_bands=[1], ch_nrad=[2, 1], n_pw=[3, 0, 5])
    raise ValueError(name)


@pytest.mark.parametrize("precision,form", [("fp64", "herk"), ("fp64", "gemm"), ("fp32", "herk"),
                                            ("bf16x3", "herk")])
@pytest.mark.parametrize("name", ["pw_only", "mt_only_q", "one_band", "max_bands"])
def test_degenerate_shapes(name, precision, form):
    import paper_1003_0524_amd as lib
    cfg = _cfg(name)
    print(f"[degenerate] {name} {precision} {form}", flush=True)
    E, D, C = synth.coulomb_blocks(cfg)
    # the GEMM form runs unbatched (one launch of each kernel per pair), the HERK forms batched
    batched = form != "gemm"
    if form == "gemm" and max(cfg.n_bands) > 64:
        # the batched GEMM form (persistent tile kernel) stops at 64 bands
        with pytest.raises(lib.ExchangeError) as e:
            lib.Exchange(cfg.n_bands, cfg.n_pw, cfg.ch_nrad, cfg.n_occ, E, D, C, w_q=cfg.weights_q(),
                         precision=precision, form=form, batched=True)
        assert e.value.status == -6
    ex = lib.Exchange(cfg.n_bands, cfg.n_pw, cfg.ch_nrad, cfg.n_occ, E, D, C, w_q=cfg.weights_q(),
                      precision=precision, form=form, batched=batched)
    Vs = [V.cpu().numpy() for V in ex.matrix_all([torch.from_numpy(synth.m_all(cfg, k)).cuda()
                                                  for k in range(cfg.n_k)])]
    e_gpu = ex.energy()
    plan = ex.accumulation_plan()
    ex.close()
    v = [vx.assemble_v(E[q], D, C) for q in range(cfg.n_q)]
    for k in range(cfg.n_k):
        blocks = [synth.m_block(cfg, k, q) for q in range(cfg.n_q)]
        ref = vx.vx_k(blocks, v, cfg.weights_q())
        err = pr.normwise_error(Vs[k], ref)
        assert np.array_equal(Vs[k], Vs[k].conj().T)
        if precision == "fp64":
            assert err <= 1e-10, (name, k, err)
        else:
            L = [chol.cholesky(a) for a in v]
            pred = pr.normwise_error(pr.vx_k_emulated(blocks, L, cfg.weights_q(), precision, cfg.n_s, plan), ref)
            assert err <= 4.0 * pred + 1e-12, (name, k, err, pred)
    e_dir = vx.energy_direct(cfg, lambda k, q: synth.m_block(cfg, k, q), v)
    assert e_gpu == pytest.approx(e_dir, rel=1e-10 if precision == "fp64" else 1e-5)
