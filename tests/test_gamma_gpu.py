"""GPU parity of the Gamma-point term (exchange_gamma_term) against the oracle.

Bars: the lattice sum to 1e-12 relative and its term count exactly (FP64 sums of
the same terms in another order; a lattice point within 1e-12 of the sphere
|p| = q0 would be a boundary case, and none of these lattices has one); C to
1e-12 of the magnitude of its two terms; with the term applied, V(k) against
the oracle's V(k) - C on the occupied diagonal to the FP64 bar of the other
parity tests (1e-10 normwise), every off-diagonal element bitwise unchanged,
and the energy shifted by -C n_occ sum_k w_k.
"""
import math
import sys

import numpy as np
import pytest

import synth
from oracle import gamma as og
from oracle import vx

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _ex(cfg, precision="fp64"):
    import paper_1003_0524_amd as lib
    E, D, C = synth.coulomb_blocks(cfg)
    return lib.Exchange(cfg.n_bands, cfg.n_pw, cfg.ch_nrad, cfg.n_occ, E, D, C,
                        w_q=cfg.weights_q(), precision=precision, form="herk", batched=True)


CASES = [
    ("small", None, (2, 2, 2), 0.05),                           # the small workload's own lattice and mesh
    ("small", np.array([[1.0, 0.2, 0.1], [0.3, 0.9, -0.2], [0.0, 0.4, 1.3]]), (2, 3, 5), 0.02),   # skewed
    ("small", 2.0 * math.pi / 10.0 * np.eye(3), (4, 4, 4), 0.05),
    ("c2", None, (4, 4, 4), 0.005),                             # Si-like fcc, the paper's beta
    ("small", 2.0 * math.pi * np.linalg.inv(synth._hex(6.14, 9.84)).T, (6, 6, 4), 0.005),   # ZnO-like hexagonal
]


@pytest.mark.parametrize("name,recip,mesh,beta", CASES)
def test_gamma_term_matches_oracle(name, recip, mesh, beta):
    cfg = synth.make_config(name)
    B = cfg.recip() if recip is None else recip
    _say(f"[gamma] {name} mesh={mesh} beta={beta}")
    ex = _ex(cfg)
    try:
        C = ex.gamma_term(B, mesh, beta, apply=False)
        ms, nterm = ex.gamma_kernel_ms()
        C2 = ex.gamma_term(B, mesh, beta, apply=False)
    finally:
        ex.close()
    q0 = og.q0_of_beta(beta)
    so, co = og.lattice_sum(B, mesh, beta, q0)
    pref = 4.0 * math.pi / (int(np.prod(mesh)) * og.cell_volume(B))
    Co = og.integral_term(beta, q0) - pref * so
    _say(f"[gamma] C={C!r} oracle={Co!r} terms={nterm} oracle terms={co} kernel {ms:.4f} ms")
    assert nterm == co
    assert C2 == C                                              # fixed summation order
    assert abs(C - Co) <= 1e-12 * (og.integral_term(beta, q0) + pref * so)


def test_gamma_shift_applied_to_matrix_and_energy():
    cfg = synth.make_config("small")
    B, mesh, beta = cfg.recip(), (2, 2, 2), 0.05
    _say("[gamma] shift small fp64")
    ex = _ex(cfg)
    try:
        Ms = [torch.from_numpy(synth.m_all(cfg, k, np.complex128)).cuda() for k in range(cfg.n_k)]
        V0 = [V.cpu().numpy() for V in ex.matrix_all(Ms)]
        E0 = ex.energy()
        C = ex.gamma_term(B, mesh, beta, apply=True)
        V1 = [V.cpu().numpy() for V in ex.matrix_all(Ms)]
        E1 = ex.energy()
        ex.gamma_term(B, mesh, beta, apply=False)
        V2 = [V.cpu().numpy() for V in ex.matrix_all(Ms)]
    finally:
        ex.close()
    Eb, Db, Cb = synth.coulomb_blocks(cfg)
    v = [vx.assemble_v(Eb[q], Db, Cb) for q in range(cfg.n_q)]
    wk = np.full(cfg.n_k, 1.0 / cfg.n_k)
    for k in range(cfg.n_k):
        Vo = og.apply_gamma(vx.vx_k([synth.m_block(cfg, k, q) for q in range(cfg.n_q)], v, cfg.weights_q()),
                            cfg.n_occ, C)
        assert np.max(np.abs(V1[k] - Vo)) <= 1e-10 * np.max(np.abs(Vo))
        off = ~np.eye(V1[k].shape[0], dtype=bool)
        assert np.array_equal(V1[k][off], V0[k][off])
        assert np.array_equal(V2[k], V0[k])                     # apply=0 removes the shift
    assert E1 - E0 == pytest.approx(-C * cfg.n_occ * float(np.sum(wk)), rel=1e-9, abs=1e-12 * abs(E0))


def test_gamma_term_rejects_bad_arguments():
    cfg = synth.make_config("small")
    import paper_1003_0524_amd as lib
    ex = _ex(cfg)
    try:
        B = cfg.recip()
        for args in [(B, (2, 2, 2), 0.0), (B, (2, 2, 2), 1.0), (B, (0, 2, 2), 0.05),
                     (np.array([[1.0, 0, 0], [2.0, 0, 0], [0, 0, 1.0]]), (2, 2, 2), 0.05),
                     (B, (2, 2, 2), 1e-9)]:
            with pytest.raises(lib.ExchangeError) as e:
                ex.gamma_term(*args)
            assert e.value.status == -1
        assert math.isfinite(ex.gamma_term(B, (2, 2, 2), 0.05))  # still usable after the errors
    finally:
        ex.close()
