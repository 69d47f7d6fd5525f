"""Synthetic outer iterations of the learned-extrapolator workload (CPU).

Pins: the occupied bases stay orthonormal and P is a rank-n_occ projector; the
exchange matrix computed from the mixed projections equals the P-weighted sum
of reference-band Gram terms (V^x is linear in P), evaluated independently of
the mixing.
"""
import numpy as np

import synth
import synth.scf as scf
from oracle import vx


def test_occupied_bases_orthonormal_and_projectors():
    cfg = synth.make_config("learn")
    seq = scf.occupied_sequence(cfg, 6)
    for U in seq:
        for u in U:
            assert np.allclose(u.conj().T @ u, np.eye(cfg.n_occ), atol=1e-13)
        for P in scf.density(U):
            assert np.allclose(P @ P, P, atol=1e-13)
            assert abs(np.trace(P).real - cfg.n_occ) < 1e-12
    # the amplitude halves per step (the random coefficients scatter single steps)
    d = [np.linalg.norm(scf.density_vector(scf.density(seq[t])) - scf.density_vector(scf.density(seq[t - 1])))
         for t in range(1, 6)]
    assert d[4] < d[0] / 4 and d[3] < d[0] / 2


def test_first_slices_of_reference_projections_are_the_workload_m():
    cfg = synth.make_config("learn")
    assert np.array_equal(scf.m_ref_block(cfg, 1, 2)[:cfg.n_occ], synth.m_block(cfg, 1, 2))


def test_exchange_is_linear_in_density_matrix():
    cfg = synth.make_config("learn")
    E, D, C = synth.coulomb_blocks(cfg)
    v = [vx.assemble_v(E[q], D, C) for q in range(cfg.n_q)]
    w = cfg.weights_q()
    U = scf.occupied_sequence(cfg, 3)[2]
    P = scf.density(U)
    k = 1
    mixed = [scf.mix(scf.m_ref_block(cfg, k, q), U[scf.k_prime(cfg, k, q)]) for q in range(cfg.n_q)]
    V = vx.vx_k(mixed, v, w)
    # independent form: -sum_q w_q sum_{m,m'} P[m,m'] Mref[m]^H v Mref[m']
    nb = cfg.n_bands[k]
    ref = np.zeros((nb, nb), dtype=np.complex128)
    for q in range(cfg.n_q):
        R = scf.m_ref_block(cfg, k, q)                 # [m][n][I]
        Pk = P[scf.k_prime(cfg, k, q)]
        for m in range(R.shape[0]):
            for mp in range(R.shape[0]):
                if abs(Pk[m, mp]) < 1e-300:
                    continue
                ref -= w[q] * Pk[m, mp] * (R[m].conj() @ v[q] @ R[mp].T)
    assert np.max(np.abs(V - ref)) <= 1e-12 * np.max(np.abs(ref))
