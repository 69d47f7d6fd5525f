"""Channel blocks given per q (exc_coulomb.D / .C as arrays over q). Two distinct sets of
multipole-free blocks, alternating over the q mesh (the second: D scaled by 1.5, C turned
by a phase, so that every v(q) stays positive definite), against the oracle with each q's
own v(q): FP64 (batched HERK, unbatched GEMM) to 1e-10, bf16x3 (fused) and fp32 (block-
sparse + tile path) within 4x the predicted error. With every q pointing at the same
blocks the result is bitwise that of the q-independent call."""
import numpy as np
import pytest

import synth
from oracle import chol, precision as pr, vx

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _blocks(name):
    cfg = synth.make_config(name)
    E, D, C = synth.coulomb_blocks(cfg)
    D2 = [1.5 * d for d in D]
    C2 = [np.exp(0.7j) * c for c in C]
    D_q = [D if q % 2 == 0 else D2 for q in range(cfg.n_q)]
    C_q = [C if q % 2 == 0 else C2 for q in range(cfg.n_q)]
    return cfg, E, D, C, D_q, C_q


@pytest.mark.parametrize("precision,form,batched,fused", [("fp64", "herk", True, None),
                                                          ("fp64", "gemm", False, None),
                                                          ("bf16x3", "herk", True, "1"),
                                                          ("fp32", "herk", True, "0")])
@pytest.mark.parametrize("name", ["small", "ragged"])
def test_per_q_channel_blocks(name, precision, form, batched, fused, monkeypatch):
    import paper_1003_0524_amd as lib
    monkeypatch.delenv("EXC_FUSED_CFG", raising=False)
    if fused is None:
        monkeypatch.delenv("EXC_FUSED", raising=False)
    else:
        monkeypatch.setenv("EXC_FUSED", fused)
    cfg, E, D, C, D_q, C_q = _blocks(name)
    print(f"[per-q] {name} {precision} {form} batched={batched} fused={fused}", flush=True)
    ex = lib.Exchange(cfg.n_bands, cfg.n_pw, cfg.ch_nrad, cfg.n_occ, E, D, C, w_q=cfg.weights_q(),
                      precision=precision, form=form, batched=batched, D_q=D_q, C_q=C_q)
    Vs = [V.cpu().numpy() for V in ex.matrix_all([torch.from_numpy(synth.m_all(cfg, k)).cuda()
                                                  for k in range(cfg.n_k)])]
    plan = ex.accumulation_plan()
    ex.close()
    v = [vx.assemble_v(E[q], D_q[q], C_q[q]) for q in range(cfg.n_q)]
    v_same = [vx.assemble_v(E[q], D, C) for q in range(cfg.n_q)]
    L = [chol.cholesky(a) for a in v]
    for k in range(cfg.n_k):
        blocks = [synth.m_block(cfg, k, q) for q in range(cfg.n_q)]
        ref = vx.vx_k(blocks, v, cfg.weights_q())
        # the two sets give different results: the test sees which one the library used
        assert pr.normwise_error(vx.vx_k(blocks, v_same, cfg.weights_q()), ref) > 1e-3
        err = pr.normwise_error(Vs[k], ref)
        assert np.array_equal(Vs[k], Vs[k].conj().T)
        if precision == "fp64":
            assert err <= 1e-10, (name, k, err)
        else:
            pred = pr.normwise_error(pr.vx_k_emulated(blocks, L, cfg.weights_q(), precision, cfg.n_s, plan), ref)
            assert err <= 4.0 * pred + 1e-12, (name, k, err, pred)


def test_aliased_per_q_blocks_equal_the_shared_call(monkeypatch):
    import paper_1003_0524_amd as lib
    monkeypatch.setenv("EXC_TUNE", "0")          # the same (default) configuration for both
    cfg, E, D, C, D_q, C_q = _blocks("ragged")
    print("[per-q] ragged aliased bf16x3", flush=True)
    Ms = [torch.from_numpy(synth.m_all(cfg, k)).cuda() for k in range(cfg.n_k)]
    out = []
    for kw in ({}, {"D_q": [D] * cfg.n_q, "C_q": [C] * cfg.n_q}):
        ex = lib.Exchange(cfg.n_bands, cfg.n_pw, cfg.ch_nrad, cfg.n_occ, E, D, C, w_q=cfg.weights_q(),
                          precision="bf16x3", form="herk", batched=True, **kw)
        out.append([V.cpu().numpy() for V in ex.matrix_all(Ms)])
        ex.close()
    for a, b in zip(*out):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("precision", ["fp64", "bf16x3"])
def test_blocks_from_device_memory(precision, monkeypatch):
    """exc_coulomb.on_device = 1 (E handed over as device tensors, per-q D and C moved to the
    device): bitwise the result of the host-pointer call."""
    import paper_1003_0524_amd as lib
    monkeypatch.setenv("EXC_TUNE", "0")
    cfg, E, D, C, D_q, C_q = _blocks("ragged")
    print(f"[per-q] ragged blocks in device memory {precision}", flush=True)
    Ms = [torch.from_numpy(synth.m_all(cfg, k)).cuda() for k in range(cfg.n_k)]
    out = []
    for E_in in (E, [torch.from_numpy(e).cuda() for e in E]):
        ex = lib.Exchange(cfg.n_bands, cfg.n_pw, cfg.ch_nrad, cfg.n_occ, E_in, D, C, w_q=cfg.weights_q(),
                          precision=precision, form="herk", batched=True, D_q=D_q, C_q=C_q)
        out.append([V.cpu().numpy() for V in ex.matrix_all(Ms)])
        ex.close()
    for a, b in zip(*out):
        assert np.array_equal(a, b)
