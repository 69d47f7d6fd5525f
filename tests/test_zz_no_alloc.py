"""exchange_matrix_noalloc (the entry point for callers that cannot allocate) against
exchange_matrix on the same context and inputs: bitwise equal results (the same kernels and
reduction order), on two calls in a row, the second with a smaller input, so that the second
call finds the first one's contents in the shared scratch; and the size refusal."""
import ctypes

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _ctx(name, precision, fused):
    import paper_1003_0524_amd as lib
    cfg = synth.make_config(name)
    E, D, C = synth.coulomb_blocks(cfg)
    return cfg, lib.Exchange(cfg.n_bands, cfg.n_pw, cfg.ch_nrad, cfg.n_occ, E, D, C, w_q=cfg.weights_q(),
                             precision=precision, form="herk", batched=True)


@pytest.mark.parametrize("precision,fused", [("bf16x3", "1"), ("bf16x3", "0"), ("fp64", "0")])
def test_noalloc_equals_exchange_matrix(precision, fused, monkeypatch):
    monkeypatch.setenv("EXC_FUSED", fused)
    monkeypatch.delenv("EXC_FUSED_CFG", raising=False)
    got_ref = []
    # the larger input first (ragged, its largest k), then a smaller one (small, k = 0)
    for name, pick in (("ragged", "largest"), ("small", "first")):
        cfg, ex = _ctx(name, precision, fused)
        k = int(np.argmax(cfg.n_bands)) if pick == "largest" else 0
        print(f"[noalloc] {name} k={k} {precision} fused={fused}", flush=True)
        M = torch.from_numpy(synth.m_all(cfg, k)).cuda()
        ref = ex.matrix(k, M).clone()
        out = torch.full((cfg.n_bands[k] ** 2,), float("nan"), dtype=torch.complex128, device="cuda")
        got = ex.matrix_noalloc(k, M, out)
        torch.cuda.synchronize()
        assert torch.equal(got, ref), (name, k)
        got_ref.append(int(ex.query(10)))
        ex.close()
    assert got_ref[0] == int(fused == "1") and got_ref[1] == int(fused == "1")


def test_noalloc_refuses_a_k_beyond_its_scratch(monkeypatch):
    """FP64 block-sparse + tile path with 1024 block-sparse rows, 8 q and 8 x 128 columns:
    the workspace of one k (8 x 1024 x 1024 complex128, 128 MiB) exceeds the 64 MiB array."""
    import paper_1003_0524_amd as lib
    monkeypatch.setenv("EXC_FUSED", "0")
    cfg = synth.Config("noalloc-big", 77, 1, 8.0 * np.eye(3), np.zeros((8, 3)), n_k=1, n_occ=8,
                       n_bands=[128], ch_nrad=[9] * 128, n_pw=[4] * 8)
    E, D, C = synth.coulomb_blocks(cfg)
    ex = lib.Exchange(cfg.n_bands, cfg.n_pw, cfg.ch_nrad, cfg.n_occ, E, D, C, w_q=cfg.weights_q(),
                      precision="fp64", form="herk", batched=True)
    print(f"[noalloc] refusal: n_s={cfg.n_s} n_mb={cfg.n_mb(0)}", flush=True)
    M = torch.zeros(ex.m_elems(0), dtype=torch.complex128, device="cuda")
    out = torch.zeros(128 * 128, dtype=torch.complex128, device="cuda")
    with pytest.raises(lib.ExchangeError) as e:
        ex.matrix_noalloc(0, M, out)
    assert e.value.status == -1 and "scratch" in str(e.value)
    ex.close()
