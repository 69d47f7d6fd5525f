"""GPU parity on seeded random shapes: band counts per k, occupied bands, channel sizes
(including channels without multipole-free functions), plane waves per q and q points
drawn at random inside the ranges the library documents (up to 40 bands in the first six
cases, up to 100 in the rest), so that no tile size divides the problem. Each case goes
through the batched FP64 Cholesky form, the unbatched FP64 GEMM form (one launch of each
kernel per pair, any band count) and the batched FP32 / bf16x3 / bf16x6 forms
(autotuned), and is compared element by element with the FP64 oracle. Bars as in the
other parity tests: FP64 normwise 1e-10; reduced precision within 4x the error the error
model predicts for the context's accumulation (plus 1e-12); Hermitian mirror and real
diagonal exact. The
inversion-symmetric variant and random per-pair weights (some zero) run on the same shapes
(FP64 and bf16x3), as does M handed over in complex64, and so do the back-transform (random n_G) and the Gamma-point term
(random skewed lattice, mesh and beta).
"""
import numpy as np
import pytest

import synth
from oracle import chol, precision as pr, vx

torch = pytest.importorskip("torch")

SEEDS = list(range(12))


def _cfg(seed):
    rng = np.random.default_rng([2718, seed])
    n_k = int(rng.integers(1, 4))
    n_q = int(rng.integers(2, 6))
    n_bands = [int(x) for x in rng.integers(1, 41 if seed < 6 else 101, size=n_k)]
    n_occ = int(rng.integers(1, min(5, min(n_bands)) + 1))
    n_ch = int(rng.integers(0, 21))
    ch = [int(x) for x in rng.integers(1, 8, size=n_ch)]
    n_pw = [int(x) for x in rng.integers(0 if n_ch else 1, 131, size=n_q)]
    q = rng.uniform(0.0, 1.0, size=(n_q, 3))
    return synth.Config(f"random{seed}", 40 + seed, seed, 8.0 * np.eye(3), q, n_k=n_k, n_occ=n_occ,
                        n_bands=n_bands, ch_nrad=ch, n_pw=n_pw)


def test_shapes_are_drawn_inside_the_documented_ranges():
    for s in SEEDS:
        cfg = _cfg(s)
        assert 1 <= min(cfg.n_bands) and max(cfg.n_bands) <= 128 and cfg.n_occ <= min(cfg.n_bands)
        assert all(cfg.n_mb(q) > 0 for q in range(cfg.n_q))


@pytest.mark.gpu
@pytest.mark.parametrize("precision,form,batched", [("fp64", "herk", True), ("fp64", "gemm", False),
                                                    ("fp32", "herk", True), ("bf16x3", "herk", True),
                                                    ("bf16x6", "herk", True)])
@pytest.mark.parametrize("seed", SEEDS)
def test_random_shape_matches_oracle(seed, precision, form, batched):
    import paper_1003_0524_amd as lib
    cfg = _cfg(seed)
    print(f"[random] seed={seed} {precision} {form} batched={batched} n_b={cfg.n_bands} n_occ={cfg.n_occ} "
          f"ch={len(cfg.ch_nrad)} n_pw={cfg.n_pw}", flush=True)
    E, D, C = synth.coulomb_blocks(cfg)
    ex = lib.Exchange(cfg.n_bands, cfg.n_pw, cfg.ch_nrad, cfg.n_occ, E, D, C, w_q=cfg.weights_q(),
                      precision=precision, form=form, batched=batched)
    Vs = [V.cpu().numpy() for V in ex.matrix_all([torch.from_numpy(synth.m_all(cfg, k)).cuda()
                                                  for k in range(cfg.n_k)])]
    plan = ex.accumulation_plan()
    ex.close()
    v = [vx.assemble_v(E[q], D, C) for q in range(cfg.n_q)]
    for k in range(cfg.n_k):
        blocks = [synth.m_block(cfg, k, q) for q in range(cfg.n_q)]
        ref = vx.vx_k(blocks, v, cfg.weights_q())
        err = pr.normwise_error(Vs[k], ref)
        assert np.array_equal(Vs[k], Vs[k].conj().T)
        assert np.all(np.diag(Vs[k]).imag == 0.0)
        if precision == "fp64":
            assert err <= 1e-10, (seed, k, err)
        else:
            L = [chol.cholesky(a) for a in v]
            pred = pr.normwise_error(pr.vx_k_emulated(blocks, L, cfg.weights_q(), precision, cfg.n_s, plan), ref)
            assert err <= 4.0 * pred + 1e-12, (seed, k, err, pred)


@pytest.mark.gpu
@pytest.mark.parametrize("precision", ["fp64", "bf16x3"])
@pytest.mark.parametrize("seed", SEEDS)
def test_random_shape_inversion_variant(seed, precision):
    """The inversion-symmetric variant (real v, real bands packed two per complex column,
    odd occupied counts included) on the same shapes: FP64 1e-10 normwise against the real
    oracle; bf16x3 within 4x the emulated error of the same packed product; V real and
    exactly symmetric."""
    import paper_1003_0524_amd as lib
    cfg = _cfg(seed)
    print(f"[random] seed={seed} inversion {precision} n_b={cfg.n_bands} n_occ={cfg.n_occ}", flush=True)
    E, D, C = synth.coulomb_blocks_real(cfg)
    ex = lib.Exchange(cfg.n_bands, cfg.n_pw, cfg.ch_nrad, cfg.n_occ, E, D, C, w_q=cfg.weights_q(),
                      precision=precision, form="herk", batched=True, inversion=True)
    Vs = [V.cpu().numpy() for V in ex.matrix_all([torch.from_numpy(synth.m_all_real_packed(cfg, k)).cuda()
                                                  for k in range(cfg.n_k)])]
    plan = ex.accumulation_plan()
    ex.close()
    v = [vx.assemble_v(E[q], D, C) for q in range(cfg.n_q)]
    L = [chol.cholesky(a) for a in v]
    for k in range(cfg.n_k):
        ref = vx.vx_k([synth.m_block_real(cfg, k, q) for q in range(cfg.n_q)], v, cfg.weights_q())
        err = pr.normwise_error(Vs[k], ref)
        assert not np.any(Vs[k].imag)
        assert np.array_equal(Vs[k], Vs[k].T)
        if precision == "fp64":
            assert err <= 1e-10, (seed, k, err)
        else:
            packed = [synth.pack_real_pairs(synth.m_block_real(cfg, k, q)) for q in range(cfg.n_q)]
            pred = pr.normwise_error(pr.vx_k_emulated(packed, L, cfg.weights_q(), precision, cfg.n_s, plan).real, ref)
            assert err <= 4.0 * pred + 1e-12, (seed, k, err, pred)


@pytest.mark.gpu
@pytest.mark.parametrize("precision", ["fp64", "bf16x3"])
@pytest.mark.parametrize("seed", SEEDS)
def test_random_shape_pair_weights(seed, precision):
    """Per-pair weights (exc_desc.w_kq, the EIBZ form of the q sum) drawn at random, about a
    third of the pairs of each k at zero and left out of M(k), on the same shapes: FP64 1e-10
    normwise against the oracle's weighted sum over the kept pairs; bf16x3 within 4x the
    emulated error of that sum."""
    import paper_1003_0524_amd as lib
    cfg = _cfg(seed)
    rng = np.random.default_rng([31337, seed])
    w_kq = rng.uniform(0.05, 1.0, size=(cfg.n_k, cfg.n_q)) / cfg.n_q
    w_kq[rng.random((cfg.n_k, cfg.n_q)) < 0.35] = 0.0
    w_kq[np.arange(cfg.n_k), rng.integers(0, cfg.n_q, size=cfg.n_k)] = 0.5 / cfg.n_q   # a pair per k
    print(f"[random] seed={seed} pair weights {precision} kept={int((w_kq != 0).sum())} of {w_kq.size}",
          flush=True)
    E, D, C = synth.coulomb_blocks(cfg)
    ex = lib.Exchange(cfg.n_bands, cfg.n_pw, cfg.ch_nrad, cfg.n_occ, E, D, C, w_q=cfg.weights_q(),
                      precision=precision, form="herk", batched=True, w_kq=w_kq)
    keep = [[q for q in range(cfg.n_q) if w_kq[k, q] != 0] for k in range(cfg.n_k)]
    blocks = [[synth.m_block(cfg, k, q) for q in keep[k]] for k in range(cfg.n_k)]
    Ms = [torch.from_numpy(np.concatenate([b.ravel() for b in blocks[k]])).cuda() for k in range(cfg.n_k)]
    Vs = [V.cpu().numpy() for V in ex.matrix_all(Ms)]
    plan = ex.accumulation_plan()
    ex.close()
    v = [vx.assemble_v(E[q], D, C) for q in range(cfg.n_q)]
    L = [chol.cholesky(a) for a in v]
    for k in range(cfg.n_k):
        vk, wk = [v[q] for q in keep[k]], w_kq[k, keep[k]]
        ref = vx.vx_k(blocks[k], vk, wk)
        err = pr.normwise_error(Vs[k], ref)
        assert np.array_equal(Vs[k], Vs[k].conj().T)
        if precision == "fp64":
            assert err <= 1e-10, (seed, k, err)
        else:
            pred = pr.normwise_error(pr.vx_k_emulated(blocks[k], [L[q] for q in keep[k]], wk, precision, cfg.n_s, plan), ref)
            assert err <= 4.0 * pred + 1e-12, (seed, k, err, pred)


def _colmajor(a):
    return torch.from_numpy(np.ascontiguousarray(a.T)).cuda().T


@pytest.mark.gpu
@pytest.mark.parametrize("seed", SEEDS)
def test_random_shape_back_transform(seed):
    """Z V(k) Z^H (the back-transform to the LAPW basis) for every k of the shape, with a
    random n_G in [1, 700] per k: 1e-12 normwise against the oracle's product of its own
    V(k), Hermitian to 1e-13."""
    import paper_1003_0524_amd as lib
    from oracle import backx
    cfg = _cfg(seed)
    rng = np.random.default_rng([4242, seed])
    E, D, C = synth.coulomb_blocks(cfg)
    ex = lib.Exchange(cfg.n_bands, cfg.n_pw, cfg.ch_nrad, cfg.n_occ, E, D, C, w_q=cfg.weights_q(),
                      precision="fp64", form="herk", batched=True)
    v = [vx.assemble_v(E[q], D, C) for q in range(cfg.n_q)]
    try:
        ex.matrix_all([torch.from_numpy(synth.m_all(cfg, k)).cuda() for k in range(cfg.n_k)])
        for k in range(cfg.n_k):
            nG, nb = int(rng.integers(1, 701)), cfg.n_bands[k]
            print(f"[random] seed={seed} back-transform k={k} n_G={nG} n_b={nb}", flush=True)
            Z = rng.standard_normal((nG, nb)) + 1j * rng.standard_normal((nG, nb))
            G = ex.back_transform(k, _colmajor(Z)).cpu().numpy()
            ref = backx.back_transform(Z, vx.vx_k([synth.m_block(cfg, k, q) for q in range(cfg.n_q)], v,
                                                  cfg.weights_q()))
            assert pr.normwise_error(G, ref) <= 1e-12, (seed, k, nG)
            assert np.max(np.abs(G - G.conj().T)) <= 1e-13 * np.abs(G).max()
    finally:
        ex.close()


@pytest.mark.gpu
@pytest.mark.parametrize("seed", SEEDS)
def test_random_gamma_term(seed):
    """The Gamma-point term on a random (skewed) reciprocal lattice, mesh and beta: the
    lattice-sum term count exactly, C to 1e-12 of the magnitude of its two terms."""
    import math
    import paper_1003_0524_amd as lib
    from oracle import gamma as og
    rng = np.random.default_rng([9001, seed])
    a = rng.uniform(6.0, 12.0)
    B = 2.0 * math.pi / a * (np.eye(3) + 0.3 * rng.uniform(-1.0, 1.0, size=(3, 3)))
    mesh = tuple(int(x) for x in rng.integers(1, 7, size=3))
    beta = float(rng.uniform(0.02, 0.2))
    print(f"[random] seed={seed} gamma mesh={mesh} beta={beta:.4f}", flush=True)
    cfg = _cfg(seed)
    E, D, C = synth.coulomb_blocks(cfg)
    ex = lib.Exchange(cfg.n_bands, cfg.n_pw, cfg.ch_nrad, cfg.n_occ, E, D, C, w_q=cfg.weights_q(),
                      precision="fp64", form="herk", batched=True)
    try:
        Cg = ex.gamma_term(B, mesh, beta, apply=False)
        _, nterm = ex.gamma_kernel_ms()
    finally:
        ex.close()
    q0 = og.q0_of_beta(beta)
    so, co = og.lattice_sum(B, mesh, beta, q0)
    pref = 4.0 * math.pi / (int(np.prod(mesh)) * og.cell_volume(B))
    Co = og.integral_term(beta, q0) - pref * so
    assert nterm == co
    assert abs(Cg - Co) <= 1e-12 * (og.integral_term(beta, q0) + pref * so)


@pytest.mark.gpu
@pytest.mark.parametrize("precision", ["fp64", "bf16x3"])
@pytest.mark.parametrize("seed", SEEDS)
def test_random_shape_complex64_input(seed, precision):
    """M handed over as complex64 (as the ZnO- and SrTiO3-like workloads do): the oracle takes
    the same complex64 values widened to complex128; FP64 1e-10 normwise, bf16x3 within 4x the
    emulated error on those values."""
    import paper_1003_0524_amd as lib
    cfg = _cfg(seed)
    print(f"[random] seed={seed} complex64 {precision} n_b={cfg.n_bands}", flush=True)
    E, D, C = synth.coulomb_blocks(cfg)
    ex = lib.Exchange(cfg.n_bands, cfg.n_pw, cfg.ch_nrad, cfg.n_occ, E, D, C, w_q=cfg.weights_q(),
                      precision=precision, form="herk", batched=True)
    Vs = [V.cpu().numpy() for V in ex.matrix_all([torch.from_numpy(synth.m_all(cfg, k, np.complex64)).cuda()
                                                  for k in range(cfg.n_k)])]
    plan = ex.accumulation_plan()
    ex.close()
    v = [vx.assemble_v(E[q], D, C) for q in range(cfg.n_q)]
    L = [chol.cholesky(a) for a in v]
    for k in range(cfg.n_k):
        blocks = [synth.m_block(cfg, k, q, np.complex64).astype(np.complex128) for q in range(cfg.n_q)]
        ref = vx.vx_k(blocks, v, cfg.weights_q())
        err = pr.normwise_error(Vs[k], ref)
        assert np.array_equal(Vs[k], Vs[k].conj().T)
        if precision == "fp64":
            assert err <= 1e-10, (seed, k, err)
        else:
            pred = pr.normwise_error(pr.vx_k_emulated(blocks, L, cfg.weights_q(), precision, cfg.n_s, plan), ref)
            assert err <= 4.0 * pred + 1e-12, (seed, k, err, pred)
