"""GPU parity of the back-transform to the LAPW basis (exchange_back_transform,
Sec. III.A, eq. "APW trafo") against the oracle.

V(k) comes from the library's FP64 path; the oracle computes its own V(k) and
Z V Z^H. Bar: 1e-12 normwise (FP64 products of FP64 inputs). Sizes n_G = 1, 70,
200, 333 cover single and partial 64-row tiles; band counts 8, 13, 21 and 37 cover
partial steps of the band index. With Z = S c, c^H S c = 1, the
projection c^H V_GG c returns the library's V(k) (1e-11 of its size).
"""
import sys

import numpy as np
import pytest

import synth
from oracle import backx, precision as pr, vx

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _colmajor(a):
    return torch.from_numpy(np.ascontiguousarray(a.T)).cuda().T


def _ctx(cfg):
    import paper_1003_0524_amd as lib
    E, D, C = synth.coulomb_blocks(cfg)
    return lib.Exchange(cfg.n_bands, cfg.n_pw, cfg.ch_nrad, cfg.n_occ, E, D, C, w_q=cfg.weights_q(),
                        precision="fp64", form="herk", batched=True)


@pytest.mark.parametrize("name", ["small", "ragged"])      # ragged: 13, 37, 21 bands
def test_back_transform_matches_oracle(name):
    cfg = synth.make_config(name)
    ex = _ctx(cfg)
    ex.matrix_all([torch.from_numpy(synth.m_all(cfg, k)).cuda() for k in range(cfg.n_k)])
    E, D, C = synth.coulomb_blocks(cfg)
    v = [vx.assemble_v(E[q], D, C) for q in range(cfg.n_q)]
    rng = np.random.default_rng(11)
    try:
        for k in range(cfg.n_k):
            Vo = vx.vx_k([synth.m_block(cfg, k, q) for q in range(cfg.n_q)], v, cfg.weights_q())
            for nG in (1, 70, 200, 333):
                _say(f"[backx] k={k} n_G={nG}")
                Z = rng.standard_normal((nG, cfg.n_bands[k])) + 1j * rng.standard_normal((nG, cfg.n_bands[k]))
                G = ex.back_transform(k, _colmajor(Z)).cpu().numpy()
                ref = backx.back_transform(Z, Vo)
                assert pr.normwise_error(G, ref) <= 1e-12, (k, nG)
                assert np.max(np.abs(G - G.conj().T)) <= 1e-13 * np.abs(G).max()
    finally:
        ex.close()


def test_projection_returns_v():
    cfg = synth.make_config("small")
    ex = _ctx(cfg)
    Vs = [V.cpu().numpy() for V in ex.matrix_all([torch.from_numpy(synth.m_all(cfg, k)).cuda()
                                                  for k in range(cfg.n_k)])]
    rng = np.random.default_rng(12)
    nG, nb = 150, cfg.n_bands[0]
    x = rng.standard_normal((nG, nG)) + 1j * rng.standard_normal((nG, nG))
    S = x @ x.conj().T / nG + np.eye(nG)
    w, U = np.linalg.eigh(S)
    Q, _ = np.linalg.qr(rng.standard_normal((nG, nb)) + 1j * rng.standard_normal((nG, nb)))
    c = U @ np.diag(w ** -0.5) @ U.conj().T @ Q
    try:
        G = ex.back_transform(0, _colmajor(S @ c)).cpu().numpy()
    finally:
        ex.close()
    assert np.max(np.abs(c.conj().T @ G @ c - Vs[0])) <= 1e-11 * np.abs(Vs[0]).max()


def test_back_transform_errors():
    import paper_1003_0524_amd as lib
    cfg = synth.make_config("small")
    ex = _ctx(cfg)
    try:
        Z = _colmajor(np.ones((10, cfg.n_bands[0]), dtype=np.complex128))
        with pytest.raises(lib.ExchangeError) as e:
            ex.back_transform(0, Z)
        assert e.value.status == -5                     # V(k) not computed yet
        st = ex.lib.exchange_back_transform(ex.ctx, 0, None, 10, None, None)
        assert st == -1
    finally:
        ex.close()
