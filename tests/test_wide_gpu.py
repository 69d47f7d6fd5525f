"""GPU parity of the wide kernel (large pairs, complex64 M): every instance forced in
turn on the small and ragged workloads (one to five band tiles, channels without
multipole-free functions) and on full per-pair shapes of the ZnO-like and SrTiO3-like
workloads (their Gamma, smallest and largest mixed basis, 60 / 100 bands, N_MB up to
1399 / 2600), against the float64 oracle on the same complex64 values widened.

Bars as in test_parity: normwise error within 4x the error model's prediction for the
context's accumulation (plus 1e-12); on the full shapes also the normalised eigenvalue error
<= 1e-6 Ha; Hermitian mirror and real diagonal exact. Work items per n'' chunk, and a
complex128 call on a context fixed to a wide instance (which switches to an instance
that reads complex128), are covered too, and so are the fused instances for up to eight band
tiles at the ZnO-like shapes.
"""
import functools
import sys

import numpy as np
import pytest

import synth
from oracle import chol, precision as pr, vx
from _emulation import predicted

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

WIDE = {"fp32": [180, 186, 183, 189], "bf16x3": [181, 187, 184, 190], "bf16x6": [182, 188, 191]}
CAP = {180: 13, 181: 13, 182: 13, 183: 16, 184: 16, 186: 13, 187: 13, 188: 13, 189: 8, 190: 8, 191: 8}


@functools.lru_cache(maxsize=None)
def _work(name):
    cfg = synth.make_config(name)
    if name in ("c3", "c4"):
        nmb = np.array([cfg.n_mb(q) for q in range(cfg.n_q)])
        cfg = synth.q_slice(cfg, [0, int(nmb.argmin()), int(nmb.argmax())], n_k=1)
    E, D, C = synth.coulomb_blocks(cfg)
    v = [vx.assemble_v(E[q], D, C) for q in range(cfg.n_q)]
    m64 = [[synth.m_block(cfg, k, q, np.complex64).astype(np.complex128) for q in range(cfg.n_q)]
           for k in range(cfg.n_k)]
    refs = [vx.vx_k(m64[k], v, cfg.weights_q()) for k in range(cfg.n_k)]
    rho = max(float(np.abs(np.linalg.eigvalsh(vx.hermitian_part(r))).max()) for r in refs)
    return cfg, E, D, C, v, m64, refs, rho


@functools.lru_cache(maxsize=None)
def _factors(name):
    return [chol.cholesky(a) for a in _work(name)[4]]


def _emulated(name, mode, plan):
    cfg, E, D, C, v, m64, refs, rho = _work(name)
    return [predicted((name, k), m64[k], _factors(name), cfg.weights_q(), mode, cfg.n_s, plan)
            for k in range(cfg.n_k)]


def _run(name, precision, dt=np.complex64):
    import paper_1003_0524_amd as lib
    cfg, E, D, C, v, m64, refs, rho = _work(name)
    ex = lib.Exchange(cfg.n_bands, cfg.n_pw, cfg.ch_nrad, cfg.n_occ, E, D, C, w_q=cfg.weights_q(),
                      precision=precision, form="herk", batched=True)
    Ms = [torch.from_numpy(synth.m_all(cfg, k, np.complex64).astype(dt)).cuda() for k in range(cfg.n_k)]
    Vs = [V.cpu().numpy() for V in ex.matrix_all(Ms)]
    cid = int(ex.query(3))
    plan = ex.accumulation_plan()
    ex.close()
    return Vs, cid, plan


def _check(name, precision, Vs, plan, eig=False):
    cfg, E, D, C, v, m64, refs, rho = _work(name)
    emu = _emulated(name, precision, plan)
    for k in range(cfg.n_k):
        err = pr.normwise_error(Vs[k], refs[k])
        pred = pr.normwise_error(emu[k], refs[k])
        print(f"[wide] {name} {precision} k={k}: error {err:.3e}, emulated {pred:.3e}", flush=True)
        assert np.array_equal(Vs[k], Vs[k].conj().T) and np.all(np.diag(Vs[k]).imag == 0.0)
        assert err <= 4.0 * pred + 1e-12, (name, precision, k, err, pred)
        if eig:
            assert pr.normalised_eig_error(Vs[k], refs[k], rho) <= 1e-6


@pytest.mark.parametrize("precision", ["fp32", "bf16x3", "bf16x6"])
@pytest.mark.parametrize("name", ["small", "ragged", "c3", "c4"])
def test_wide_instance_matches_oracle(name, precision, monkeypatch):
    monkeypatch.delenv("EXC_FUSED", raising=False)
    monkeypatch.delenv("EXC_FUSED_SPLIT", raising=False)
    cfg = _work(name)[0]
    nbt = max((nb + 7) // 8 for nb in cfg.n_bands)
    for cid in WIDE[precision]:
        if CAP[cid] < nbt or (name in ("small", "ragged") and CAP[cid] == 16):
            continue
        monkeypatch.setenv("EXC_FUSED_CFG", str(cid))
        print(f"[wide] {name} {precision} instance {cid}", flush=True)
        sys.stdout.flush()
        Vs, got, plan = _run(name, precision)
        assert got == cid
        _check(name, precision, Vs, plan, eig=name in ("c3", "c4"))


@pytest.mark.parametrize("name,precision,cid,split", [("ragged", "bf16x3", 181, 1), ("ragged", "fp32", 186, 1),
                                                       ("ragged", "bf16x3", 181, 2), ("c3", "bf16x3", 181, 2),
                                                       ("c3", "fp32", 186, 2)])
def test_wide_split_items(name, precision, cid, split, monkeypatch):
    """Work items per n'' chunk (split 1) or per n'' chunk and row part (split 2: the block-sparse
    rows, then each 256-row dense block, every part in its own partial slot)."""
    monkeypatch.delenv("EXC_FUSED", raising=False)
    monkeypatch.setenv("EXC_FUSED_CFG", str(cid))
    monkeypatch.setenv("EXC_FUSED_SPLIT", str(split))
    print(f"[wide] {name} {precision} {cid} split {split}", flush=True)
    Vs, got, plan = _run(name, precision)
    assert got == cid and plan["split"] == split
    _check(name, precision, Vs, plan, eig=name == "c3")


def test_complex128_call_leaves_the_wide_instance(monkeypatch):
    monkeypatch.delenv("EXC_FUSED", raising=False)
    monkeypatch.delenv("EXC_FUSED_SPLIT", raising=False)
    monkeypatch.setenv("EXC_FUSED_CFG", "181")
    print("[wide] small bf16x3 fixed to 181, complex128 M", flush=True)
    Vs, got, plan = _run("small", "bf16x3", dt=np.complex128)
    assert got != 181
    _check("small", "bf16x3", Vs, plan)


@pytest.mark.parametrize("cid", [162, 131])
def test_fused_eight_band_tile_instances_on_the_zno_like_slice(cid, monkeypatch):
    """The fused instances for up to 8 band tiles (162: two workgroups per CU; 131: one) at the
    ZnO-like workload's full per-pair shapes (60 bands, N_MB up to 1399), complex64 M."""
    monkeypatch.delenv("EXC_FUSED", raising=False)
    monkeypatch.delenv("EXC_FUSED_SPLIT", raising=False)
    monkeypatch.setenv("EXC_FUSED_CFG", str(cid))
    print(f"[wide] c3 bf16x3 fused instance {cid}", flush=True)
    Vs, got, plan = _run("c3", "bf16x3")
    assert got == cid
    _check("c3", "bf16x3", Vs, plan, eig=True)
