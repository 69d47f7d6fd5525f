"""GPU parity of the inversion-symmetric (real) variant through the C ABI.

Real v(q) (the real parts of the synthetic blocks) and real projections, passed
as packed band pairs (exc_desc.inversion = 1). Bars: FP64 forms 1e-10 normwise
against the oracle's real V; reduced-precision modes within 4x the error the
input-rounding emulator predicts for the same packed product (plus 1e-12);
V real (Im = 0 exactly) and exactly symmetric; the energy against the oracle's
directly summed energy over the real bands; the nominal flops a quarter of the
complex count (real multiply-adds) for the real band count.
"""
import functools
import sys

import numpy as np
import pytest

import synth
from oracle import chol, precision as pr, vx

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@functools.lru_cache(maxsize=None)
def _case(name):
    cfg = synth.make_config(name)
    E, D, C = synth.coulomb_blocks_real(cfg)
    v = [vx.assemble_v(E[q], D, C) for q in range(cfg.n_q)]
    return cfg, E, D, C, v


@functools.lru_cache(maxsize=None)
def _oracle(name, k):
    cfg, E, D, C, v = _case(name)
    return vx.vx_k([synth.m_block_real(cfg, k, q) for q in range(cfg.n_q)], v, cfg.weights_q())


def _ex(name, precision, form="herk", batched=True):
    import paper_1003_0524_amd as lib
    cfg, E, D, C, v = _case(name)
    return lib.Exchange(cfg.n_bands, cfg.n_pw, cfg.ch_nrad, cfg.n_occ, E, D, C, w_q=cfg.weights_q(),
                        precision=precision, form=form, batched=batched, inversion=True)


def _run(name, precision, form="herk", batched=True):
    cfg = _case(name)[0]
    _say(f"[inversion] {name} precision={precision} form={form} batched={batched}")
    ex = _ex(name, precision, form, batched)
    Ms = [torch.from_numpy(synth.m_all_real_packed(cfg, k)).cuda() for k in range(cfg.n_k)]
    Vs = [V.cpu().numpy() for V in ex.matrix_all(Ms)]
    return cfg, ex, Vs


def _check_real_symmetric(V):
    assert not np.any(V.imag)
    assert np.array_equal(V, V.T)


@pytest.mark.parametrize("name", ["small", "ragged"])
@pytest.mark.parametrize("form,batched", [("gemm", False), ("herk", True), ("herk", False)])
def test_fp64_real_variant_matches_oracle(name, form, batched):
    cfg, ex, Vs = _run(name, "fp64", form, batched)
    ex.close()
    for k in range(cfg.n_k):
        ref = _oracle(name, k)
        assert pr.normwise_error(Vs[k], ref) <= 1e-10, (name, k)
        _check_real_symmetric(Vs[k])


@pytest.mark.parametrize("precision", ["fp32", "bf16x3", "bf16x6"])
@pytest.mark.parametrize("name", ["small", "ragged"])
def test_reduced_precision_real_variant(name, precision):
    cfg, ex, Vs = _run(name, precision)
    plan = ex.accumulation_plan()
    ex.close()
    _, E, D, C, v = _case(name)
    L = [chol.cholesky(a) for a in v]
    for k in range(cfg.n_k):
        ref = _oracle(name, k)
        packed = [synth.pack_real_pairs(synth.m_block_real(cfg, k, q)) for q in range(cfg.n_q)]
        emu = pr.vx_k_emulated(packed, L, cfg.weights_q(), precision, cfg.n_s, plan).real
        pred = pr.normwise_error(emu, ref)
        err = pr.normwise_error(Vs[k], ref)
        assert err <= 4.0 * pred + 1e-12, (name, precision, k, err, pred)
        _check_real_symmetric(Vs[k])


def test_real_variant_energy_and_accounting():
    name = "small"
    cfg, E, D, C, v = _case(name)
    _, ex, Vs = _run(name, "fp64")
    e_gpu = ex.energy()
    nominal = ex.query(1)
    ex.close()
    e_dir = vx.energy_direct(cfg, lambda k, q: synth.m_block_real(cfg, k, q), v)
    assert e_gpu == pytest.approx(e_dir, rel=1e-10)
    # the complex context of the same sizes counts 8 flops per multiply-add
    import paper_1003_0524_amd as lib
    Ec, Dc, Cc = synth.coulomb_blocks(cfg)
    exc = lib.Exchange(cfg.n_bands, cfg.n_pw, cfg.ch_nrad, cfg.n_occ, Ec, Dc, Cc, w_q=cfg.weights_q(),
                       precision="fp64", form="herk", batched=True)
    assert nominal == pytest.approx(exc.query(1) / 4.0, rel=1e-12)
    exc.close()


REAL_IDS = {"fp32": (250, 251), "bf16x3": (260, 261), "bf16x6": (270, 271)}
COMPLEX_TWIN = {250: 150, 251: 151, 260: 160, 261: 161, 270: 170, 271: 171}


@pytest.mark.parametrize("precision", ["fp32", "bf16x3", "bf16x6"])
@pytest.mark.parametrize("name", ["small", "c1"])          # (the real-factor instances hold <= 3 band tiles)
def test_real_factor_instances(name, precision, monkeypatch):
    """Each real-factor instance (products with the zero imaginary parts of the factor left
    out) gives bitwise the result of its general twin on the same real inputs."""
    monkeypatch.delenv("EXC_FUSED", raising=False)
    monkeypatch.delenv("EXC_TUNE_CACHE", raising=False)
    cfg = _case(name)[0]
    for cid in REAL_IDS[precision]:
        out = {}
        for use in (cid, COMPLEX_TWIN[cid]):
            monkeypatch.setenv("EXC_FUSED_CFG", str(use))
            _, ex, Vs = _run(name, precision)
            assert int(ex.query(3)) == use
            ex.close()
            out[use] = Vs
        for k in range(cfg.n_k):
            assert np.array_equal(out[cid][k], out[COMPLEX_TWIN[cid]][k]), (name, precision, cid, k)


def test_autotuner_prefers_real_factor_instances(monkeypatch):
    monkeypatch.delenv("EXC_FUSED_CFG", raising=False)
    monkeypatch.delenv("EXC_FUSED", raising=False)
    monkeypatch.delenv("EXC_TUNE_CACHE", raising=False)
    _, ex, _ = _run("small", "bf16x3")
    chosen = int(ex.query(3))
    ex.close()
    # a real context may run any fused instance that fits (all are exact for a real factor);
    # the default choice before tuning is a real-factor one
    import paper_1003_0524_amd as lib
    cfg, E, D, C, v = _case("small")
    ex2 = lib.Exchange(cfg.n_bands, cfg.n_pw, cfg.ch_nrad, cfg.n_occ, E, D, C, w_q=cfg.weights_q(),
                       precision="bf16x3", form="herk", batched=True, inversion=True)
    assert int(ex2.query(3)) in REAL_IDS["bf16x3"]
    ex2.close()
    assert chosen > 0
