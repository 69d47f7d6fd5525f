"""The block-sparse kernel of the Cholesky/HERK form with each of its column counts per
wavefront (EXC_SPARSE_NCW = 1, 2, 4; the library picks one from the LDS a column needs).

Workloads: `ragged` (channel runs of 0-6 terms, column counts per pair 65 / 185 / 105, so
the last workgroup of a pair is partly idle for every count) and a slice of the Si-like
workload (q = 0, 1, 2 of its first k: channels of up to 10 radial functions, so runs of 9
terms take two rounds of eight loads), each with complex128 M (rows staged straight into
LDS) and complex64 M (staged through registers). FP64: the batched path against the
oracle, <= 1e-10 normwise. bf16x3 on the block-sparse + tile path (the kernel also packs the
dense rows there): the same bits for every column count, since each column's arithmetic
does not depend on how columns are grouped.
"""
import functools

import numpy as np
import pytest

import synth
from oracle import precision as pr, vx

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DTYPES = {"c128": np.complex128, "c64": np.complex64}


@functools.lru_cache(maxsize=None)
def _case(name):
    if name == "c2-slice":
        cfg = synth.q_slice(synth.make_config("c2"), [0, 1, 2], n_k=1)
    else:
        cfg = synth.make_config(name)
    E, D, C = synth.coulomb_blocks(cfg)
    return cfg, E, D, C


@functools.lru_cache(maxsize=None)
def _oracle(name, dt, k):
    cfg, E, D, C = _case(name)
    v = [vx.assemble_v(E[q], D, C) for q in range(cfg.n_q)]
    m = [synth.m_block(cfg, k, q, DTYPES[dt]).astype(np.complex128) for q in range(cfg.n_q)]
    return vx.vx_k(m, v, cfg.weights_q())


def _run(name, precision, dt, ncw, monkeypatch):
    import paper_1003_0524_amd as lib
    monkeypatch.setenv("EXC_SPARSE_NCW", str(ncw))
    monkeypatch.setenv("EXC_FUSED", "0")             # reduced precision: block-sparse + tile path
    monkeypatch.delenv("EXC_FUSED_CFG", raising=False)
    cfg, E, D, C = _case(name)
    print(f"[sparse-ncw] {name} {precision} {dt} ncw={ncw}", flush=True)
    ex = lib.Exchange(cfg.n_bands, cfg.n_pw, cfg.ch_nrad, cfg.n_occ, E, D, C, w_q=cfg.weights_q(),
                      precision=precision, form="herk", batched=True)
    Ms = [torch.from_numpy(synth.m_all(cfg, k, DTYPES[dt])).cuda() for k in range(cfg.n_k)]
    Vs = [V.cpu().numpy().copy() for V in ex.matrix_all(Ms)]
    torch.cuda.synchronize()
    ex.close()
    return cfg, Vs


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("ncw", [1, 2, 4])
@pytest.mark.parametrize("name", ["ragged", "c2-slice"])
def test_fp64_every_column_count_matches_oracle(name, ncw, dt, monkeypatch):
    cfg, Vs = _run(name, "fp64", dt, ncw, monkeypatch)
    for k in range(cfg.n_k):
        err = pr.normwise_error(Vs[k], _oracle(name, dt, k))
        assert err <= 1e-10, (name, ncw, dt, k, err)


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("name", ["ragged", "c2-slice"])
def test_packed_path_same_bits_for_every_column_count(name, dt, monkeypatch):
    ref = None
    for ncw in (1, 2, 4):
        cfg, Vs = _run(name, "bf16x3", dt, ncw, monkeypatch)
        if ref is None:
            ref = Vs
            for k in range(cfg.n_k):          # (and the result is the exchange matrix)
                assert pr.normwise_error(Vs[k], _oracle(name, dt, k)) <= 1e-4
            continue
        for k in range(cfg.n_k):
            assert np.array_equal(Vs[k], ref[k]), (name, dt, ncw, k)
