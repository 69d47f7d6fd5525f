"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test is chosen so that a plausible mistake in the oracle (a dropped term,
a wrong sign, a wrong index, a transposed or conjugated operand, a misplaced
Coulomb block) fails at least one of them.
"""
import json
import math
import os

import numpy as np
import pytest

import synth
from oracle import brute, chol, transform, vx

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rand_hpd(rng, n, shift=0.5):
    x = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    return x @ x.conj().T / n + shift * np.eye(n)


def _rand_m(rng, nocc, nb, nmb):
    return rng.standard_normal((nocc, nb, nmb)) + 1j * rng.standard_normal((nocc, nb, nmb))


def _cfg_data(name):
    cfg = synth.make_config(name)
    E, D, C = synth.coulomb_blocks(cfg)
    v = [vx.assemble_v(E[q], D, C) for q in range(cfg.n_q)]
    return cfg, E, D, C, v


# --------------------------------------------------------------------------
# generator
# --------------------------------------------------------------------------
def test_splitmix64_published_outputs():
    g = json.load(open(os.path.join(GOLD, "splitmix64_seed0.json")))
    got = [synth.sm_int(0, i) for i in range(5)]
    assert got == [int(h, 16) for h in g["outputs_hex"]]
    arr = synth.splitmix64_stream(0, 0, 5)
    assert [int(x) for x in arr] == got


def test_m_block_deterministic_and_counter_addressable():
    cfg = synth.make_config("small")
    a = synth.m_block(cfg, 1, 3)
    b = synth.m_block(cfg, 1, 3)
    assert np.array_equal(a, b)
    # element (n'', n, I) is Box-Muller pair e = (n'' nb + n) N_MB + I of the substream
    nb, nmb = cfg.n_bands[1], cfg.n_mb(3)
    e = (2 * nb + 5) * nmb + 7
    z0, z1 = synth.normal_pairs(synth.stream_seed(cfg.seed, cfg.tag, 1, 3), e, 1)
    want = (z0[0] + 1j * z1[0]) * math.exp(-0.1 * 7 / nmb)
    assert a[2, 5, 7] == pytest.approx(want, rel=1e-15)
    # Box-Muller normals: mean ~0, variance ~1
    cfg2 = synth.make_config("c2")
    big = synth.m_block(cfg2, 0, 0)
    big = big / np.exp(-0.1 * np.arange(cfg2.n_mb(0)) / cfg2.n_mb(0))
    for part in (big.real, big.imag):
        assert abs(part.mean()) < 0.01 and abs(part.var() - 1.0) < 0.01


def test_coulomb_blocks_pd_and_structure():
    cfg, E, D, C, v = _cfg_data("ragged")
    for q in range(cfg.n_q):
        assert np.allclose(v[q], v[q].conj().T, atol=0, rtol=0)
        assert np.linalg.eigvalsh(v[q])[0] > 0
        assert v[q].shape[0] == cfg.n_mb(q)


# --------------------------------------------------------------------------
# the definition
# --------------------------------------------------------------------------
def test_hand_fixture_2x2():
    g = json.load(open(os.path.join(GOLD, "vx_hand_2x2.json")))
    v = np.array(g["v_re"]) + 1j * np.array(g["v_im"])
    m = (np.array(g["M_re"]) + 1j * np.array(g["M_im"]))[None]   # [n_occ=1][n_b][N_MB]
    want = np.array(g["V_re"]) + 1j * np.array(g["V_im"])
    assert np.allclose(vx.vx_k([m], [v], [1.0]), want, atol=1e-15)
    assert np.allclose(brute.brute_vx([m], [v], [1.0]), want, atol=1e-15)


def test_scalar_case_closed_form():
    # n_b = n_occ = N_q = N_MB = 1: V = -w |m|^2 v
    m = np.array([[[1.0 + 2.0j]]])
    assert vx.vx_k([m], [np.array([[3.0 + 0j]])], [0.25])[0, 0] == pytest.approx(-0.25 * 5 * 3)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_brute_force_matches_oracle(seed):
    rng = np.random.default_rng(seed)
    nq, nocc, nb = 3, 2, 4
    sizes = [12, 7, 10]
    mb = [_rand_m(rng, nocc, nb, n) for n in sizes]
    vl = [_rand_hpd(rng, n) for n in sizes]
    w = rng.uniform(0.1, 1.0, size=nq)
    a = vx.vx_k(mb, vl, w)
    b = brute.brute_vx(mb, vl, w)
    assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(b))


def test_brute_force_matches_oracle_on_block_config():
    cfg, E, D, C, v = _cfg_data("tiny")
    w = cfg.weights_q()
    for k in range(cfg.n_k):
        mb = [synth.m_block(cfg, k, q) for q in range(cfg.n_q)]
        a = vx.vx_k(mb, v, w)
        b = brute.brute_vx(mb, v, w)
        assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(b))


def test_hermitian_and_negative_semidefinite():
    cfg, E, D, C, v = _cfg_data("small")
    w = cfg.weights_q()
    for k in range(cfg.n_k):
        V = vx.vx_k([synth.m_block(cfg, k, q) for q in range(cfg.n_q)], v, w)
        nrm = np.max(np.abs(V))
        assert np.max(np.abs(V - V.conj().T)) <= 1e-14 * nrm
        lam = np.linalg.eigvalsh(vx.hermitian_part(V))
        assert lam[-1] <= 1e-12 * nrm


def test_identity_coulomb_gives_gram_matrix():
    # v = I: V = -sum_q w_q sum_n'' sum_I conj(M[n''][n][I]) M[n''][n'][I]  (written as einsum)
    rng = np.random.default_rng(5)
    mb = [_rand_m(rng, 3, 5, n) for n in (9, 11)]
    w = np.array([0.3, 0.7])
    got = vx.vx_k(mb, [np.eye(9), np.eye(11)], w)
    want = -sum(wq * np.einsum("pni,pmi->nm", m.conj(), m) for wq, m in zip(w, mb))
    assert np.allclose(got, want, rtol=1e-14, atol=1e-13)


def test_rank_one_coulomb():
    rng = np.random.default_rng(6)
    nb, nocc, n = 6, 2, 8
    u = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    m = _rand_m(rng, nocc, nb, n)
    V = vx.vx_k([m], [np.outer(u, u.conj())], [1.0])
    # V_{nn'} = -sum_n'' conj(u^H a_n) (u^H a_n'),  a_n = m[n''][n]
    c = np.einsum("i,pni->pn", u.conj(), m)
    want = -np.einsum("pn,pm->nm", c.conj(), c)
    assert np.allclose(V, want, rtol=1e-13, atol=1e-12)
    assert np.linalg.matrix_rank(V, tol=1e-9 * np.abs(V).max()) <= nocc


def test_scaling_and_linearity():
    rng = np.random.default_rng(7)
    mb = [_rand_m(rng, 2, 4, 6) for _ in range(2)]
    v1 = [_rand_hpd(rng, 6) for _ in range(2)]
    v2 = [_rand_hpd(rng, 6) for _ in range(2)]
    w = np.array([0.25, 0.75])
    V1 = vx.vx_k(mb, v1, w)
    c = 0.3 - 1.7j
    assert np.allclose(vx.vx_k([c * m for m in mb], v1, w), abs(c) ** 2 * V1, rtol=1e-13)
    V12 = vx.vx_k(mb, [a + 2 * b for a, b in zip(v1, v2)], w)
    assert np.allclose(V12, V1 + 2 * vx.vx_k(mb, v2, w), rtol=1e-13, atol=1e-12)
    Vw = vx.vx_k(mb, v1, 2 * w)
    assert np.allclose(Vw, 2 * V1, rtol=1e-14)
    # q sum is additive: one q at a time
    parts = vx.vx_k(mb[:1], v1[:1], w[:1]) + vx.vx_k(mb[1:], v1[1:], w[1:])
    assert np.allclose(parts, V1, rtol=1e-14, atol=1e-13)


def test_block_diagonal_coulomb_is_sum_of_blocks():
    rng = np.random.default_rng(8)
    a, b = _rand_hpd(rng, 4), _rand_hpd(rng, 5)
    v = np.zeros((9, 9), complex)
    v[:4, :4], v[4:, 4:] = a, b
    m = _rand_m(rng, 2, 3, 9)
    got = vx.vx_k([m], [v], [1.0])
    want = vx.vx_k([m[..., :4]], [a], [1.0]) + vx.vx_k([m[..., 4:]], [b], [1.0])
    assert np.allclose(got, want, rtol=1e-13, atol=1e-12)


# --------------------------------------------------------------------------
# sparse (transformed) MPB  ==  dense untransformed MPB
# --------------------------------------------------------------------------
def _physical_untransformed(rng, ch_nrad, n_pw):
    """An untransformed Coulomb matrix obeying the paper's electrostatics.

    Each MT function i of channel c has a multipole moment mu_i. Outside its
    own channel it interacts only through that moment (the field outside the
    sphere of a function is fixed by its multipole moment), so every coupling
    of function i with anything outside channel c is mu_i * f(c, .). Inside the
    channel there is an arbitrary onsite block.
    """
    n_ch = len(ch_nrad)
    n_mt = int(sum(ch_nrad))
    n = n_mt + n_pw
    mus = [rng.standard_normal(b) for b in ch_nrad]
    # external field model: a PD matrix over [channel multipoles, PWs]
    ext = _rand_hpd(rng, n_ch + n_pw, shift=1.0)
    # expansion of each original function onto the external model:
    # function (c, i) -> mu_i * e_c ; plane wave p -> e_{n_ch + p}
    X = np.zeros((n, n_ch + n_pw))
    off = 0
    for c, b in enumerate(ch_nrad):
        X[off:off + b, c] = mus[c]
        off += b
    for p in range(n_pw):
        X[n_mt + p, n_ch + p] = 1.0
    v = X @ ext @ X.T
    off = 0
    for c, b in enumerate(ch_nrad):      # onsite (short-range) part, channel-local
        v[off:off + b, off:off + b] += _rand_hpd(rng, b, shift=0.2)
        off += b
    return 0.5 * (v + v.conj().T), mus


def test_multipole_rotation_makes_fig1_sparsity():
    rng = np.random.default_rng(11)
    ch = [3, 1, 4, 2, 2]
    n_pw = 6
    v_orig, mus = _physical_untransformed(rng, ch, n_pw)
    n_d = len(ch) + n_pw
    T = transform.sparse_order_unitary(ch, mus, n_d)
    v_s = T @ v_orig @ T.T
    # allowed nonzeros: D_c blocks, C_c couplings, the dense block
    n_s = sum(b - 1 for b in ch)
    mask = np.zeros_like(v_s, dtype=bool)
    off = 0
    for c, b in enumerate(ch):
        mask[off:off + b - 1, off:off + b - 1] = True
        mask[off:off + b - 1, n_s + c] = True
        mask[n_s + c, off:off + b - 1] = True
        off += b - 1
    mask[n_s:, n_s:] = True
    scale = np.abs(v_s).max()
    assert np.abs(v_s[~mask]).max() <= 1e-13 * scale
    # and the multipole-free functions really are coupled to their own multipole function
    assert np.abs(v_s[0:2, n_s + 0]).max() > 1e-3 * scale


def test_dense_equals_sparse_transformed():
    rng = np.random.default_rng(12)
    ch = [3, 1, 4, 2, 2]
    n_pw = 6
    v_orig, mus = _physical_untransformed(rng, ch, n_pw)
    n_d = len(ch) + n_pw
    T = transform.sparse_order_unitary(ch, mus, n_d)
    v_s = T @ v_orig @ T.T
    # cut v_s into the library's blocks and re-assemble with the oracle's layout
    n_s = sum(b - 1 for b in ch)
    D, C = [], []
    off = 0
    for c, b in enumerate(ch):
        D.append(v_s[off:off + b - 1, off:off + b - 1])
        C.append(v_s[off:off + b - 1, n_s + c])
        off += b - 1
    v_blocks = vx.assemble_v(v_s[n_s:, n_s:], D, C)
    m_s = _rand_m(rng, 2, 5, v_orig.shape[0])
    m_orig = np.einsum("ji,pnj->pni", T, m_s)      # m_orig = T^T m_s
    V_dense = vx.vx_k([m_orig], [v_orig], [1.0])
    V_sparse = vx.vx_k([m_s], [v_blocks], [1.0])
    assert np.max(np.abs(V_dense - V_sparse)) <= 1e-12 * np.max(np.abs(V_dense))


def test_two_function_rotation_is_paper_formula():
    mu1, mu2 = 0.7, -1.9
    R = transform.two_function_rotation(mu1, mu2)
    assert np.allclose(R @ R.T, np.eye(2), atol=1e-15)
    mom = R @ np.array([mu1, mu2])
    assert mom[0] == pytest.approx(math.hypot(mu1, mu2))
    assert abs(mom[1]) < 1e-15
    H = transform.householder_rotation(np.array([mu1, mu2]), 0)
    # same multipole function; multipole-free function equal up to sign
    assert np.allclose(H[0], R[0], atol=1e-15)
    assert np.allclose(np.abs(H[1]), np.abs(R[1]), atol=1e-15)


@pytest.mark.parametrize("n", [1, 2, 3, 10])
def test_householder_rotation_leaves_one_moment(n):
    rng = np.random.default_rng(n)
    mu = rng.standard_normal(n)
    U = transform.householder_rotation(mu, n - 1)
    assert np.allclose(U @ U.T, np.eye(n), atol=1e-14)
    mom = transform.moments(U, mu)
    assert np.allclose(mom[:-1], 0.0, atol=1e-14)
    assert abs(mom[-1]) == pytest.approx(np.linalg.norm(mu))


# --------------------------------------------------------------------------
# energy and Cholesky re-arrangement
# --------------------------------------------------------------------------
def test_energy_trace_equals_direct_sum():
    cfg, E, D, C, v = _cfg_data("small")
    w = cfg.weights_q()
    Vs = [vx.vx_k([synth.m_block(cfg, k, q) for q in range(cfg.n_q)], v, w) for k in range(cfg.n_k)]
    rho = [vx.default_rho(cfg.n_bands[k], cfg.n_occ) for k in range(cfg.n_k)]
    e_tr = vx.energy_trace(Vs, cfg.weights_k(), rho)
    e_dir = vx.energy_direct(cfg, lambda k, q: synth.m_block(cfg, k, q), v)
    assert e_tr == pytest.approx(e_dir, rel=1e-12)
    assert e_tr < 0


def test_cholesky_factor_and_herk_form():
    cfg, E, D, C, v = _cfg_data("ragged")
    for q in range(cfg.n_q):
        L = chol.cholesky(v[q])
        assert np.allclose(np.triu(L, 1), 0)
        assert np.all(np.diag(L).real > 0) and np.allclose(np.diag(L).imag, 0)
        assert np.max(np.abs(L @ L.conj().T - v[q])) <= 1e-14 * np.max(np.abs(v[q])) * 10
    w = cfg.weights_q()
    for k in range(cfg.n_k):
        mb = [synth.m_block(cfg, k, q) for q in range(cfg.n_q)]
        a = vx.vx_k(mb, v, w)
        b = chol.vx_k_cholesky(mb, v, w)
        assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(a))
