"""GPU parity at the full per-pair shapes of the ZnO-like and SrTiO3-like workloads.

The whole workloads (144 and 216 q points, 21 and 20 irreducible k) are too large
for the oracle, so each is sliced to three of its q points -- Gamma, the smallest
and the largest mixed basis -- and its first irreducible k, with the workload's own
M(k,q) and v(q) at those points (uneven N_MB up to 1399 and 2600, 60 and 100 bands,
18 and 20 occupied, complex64 M). The batched path runs as the benchmark runs it:
one persistent launch in a HIP graph with the autotuned configuration (on these
shapes: the wide-band fused instances or the block-sparse + tile path). Bars as in
test_parity: FP64 <= 1e-10 normwise, reduced precision within 4x the error the error
model predicts for the context's accumulation, and <= 1e-6 Ha on the normalised
eigenvalues in every reduced-precision mode (bf16x3, headlined on these workloads,
included).
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


@functools.lru_cache(maxsize=None)
def _slice(name):
    cfg = synth.make_config(name)
    nmb = np.array([cfg.n_mb(q) for q in range(cfg.n_q)])
    sl = synth.q_slice(cfg, [0, int(nmb.argmin()), int(nmb.argmax())], n_k=1)
    E, D, C = synth.coulomb_blocks(sl)
    return sl, E, D, C


@functools.lru_cache(maxsize=None)
def _m(name):
    sl = _slice(name)[0]
    return [synth.m_block(sl, 0, q, np.complex64).astype(np.complex128) for q in range(sl.n_q)]


@functools.lru_cache(maxsize=None)
def _oracle(name):
    sl, E, D, C = _slice(name)
    v = [vx.assemble_v(E[q], D, C) for q in range(sl.n_q)]
    return vx.vx_k(list(_m(name)), v, sl.weights_q())


@functools.lru_cache(maxsize=None)
def _factors(name, real=False):
    sl, E, D, C = _slice(name)
    if real:
        E, D, C = ([x.real for x in E], [x.real for x in D], [x.real for x in C])
    return [chol.cholesky(vx.assemble_v(E[q], D, C)) for q in range(sl.n_q)]


def _emulated(name, mode, plan):
    sl = _slice(name)[0]
    return predicted((name, 0), list(_m(name)), _factors(name), sl.weights_q(), mode, sl.n_s, plan)


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3", "bf16x6"])
@pytest.mark.parametrize("name", ["c3", "c4"])
def test_full_shape_slice(name, precision):
    import paper_1003_0524_amd as lib
    sl, E, D, C = _slice(name)
    print(f"[full-shape] {sl.name} {precision} N_MB={[sl.n_mb(q) for q in range(sl.n_q)]}", flush=True)
    sys.stdout.flush()
    ex = lib.Exchange(sl.n_bands, sl.n_pw, sl.ch_nrad, sl.n_occ, E, D, C, w_q=sl.weights_q(),
                      precision=precision, form="herk", batched=True)
    M = torch.from_numpy(synth.m_all(sl, 0, np.complex64)).cuda()
    V = ex.matrix_all([M])[0]
    torch.cuda.synchronize()
    got = V.cpu().numpy()
    cfg_id = int(ex.query(3))
    plan = ex.accumulation_plan()
    ex.close()
    ref = _oracle(name)
    err = pr.normwise_error(got, ref)
    print(f"[full-shape] config {cfg_id}: normwise error {err:.3e}", flush=True)
    assert np.array_equal(got, got.conj().T) and np.all(np.diag(got).imag == 0.0)
    if precision == "fp64":
        assert err <= 1e-10, (name, err)
        return
    pred = pr.normwise_error(_emulated(name, precision, plan), ref)
    print(f"[full-shape] emulated {pred:.3e}, ratio {err / pred:.2f}", flush=True)
    assert err <= 4.0 * pred + 1e-12, (name, precision, cfg_id, err, pred)
    rho = np.abs(np.linalg.eigvalsh(vx.hermitian_part(ref))).max()
    assert pr.normalised_eig_error(got, ref, rho) <= 1e-6


@pytest.mark.parametrize("name,precision", [("c3", "fp64"), ("c3", "fp32"), ("c3", "bf16x3"),
                                            ("c4", "fp64"), ("c4", "bf16x3")])
def test_full_shape_inversion_variant(name, precision):
    """The inversion-symmetric variant at the ZnO-like and SrTiO3-like per-pair shapes (real
    parts of the slice's v and projections; 18 / 20 real bands packed into 9 / 10 columns,
    60 / 100 bands): FP64 1e-10, reduced precision within 4x the predicted error and
    <= 1e-6 Ha on the normalised eigenvalues."""
    import paper_1003_0524_amd as lib
    sl, E, D, C = _slice(name)
    Er, Dr, Cr = ([np.ascontiguousarray(x.real) for x in E], [np.ascontiguousarray(x.real) for x in D],
                  [np.ascontiguousarray(x.real) for x in C])
    mr = [np.ascontiguousarray(m.real) for m in _m(name)]
    print(f"[full-shape] {name} inversion {precision}", flush=True)
    ex = lib.Exchange(sl.n_bands, sl.n_pw, sl.ch_nrad, sl.n_occ, Er, Dr, Cr, w_q=sl.weights_q(),
                      precision=precision, form="herk", batched=True, inversion=True)
    M = torch.from_numpy(np.concatenate([synth.pack_real_pairs(m).ravel() for m in mr])).cuda()
    got = ex.matrix_all([M])[0].cpu().numpy()
    cfg_id = int(ex.query(3))
    plan = ex.accumulation_plan()
    ex.close()
    v = [vx.assemble_v(Er[q], Dr, Cr) for q in range(sl.n_q)]
    ref = vx.vx_k(mr, v, sl.weights_q())
    err = pr.normwise_error(got, ref)
    print(f"[full-shape] config {cfg_id}: normwise error {err:.3e}", flush=True)
    assert not np.any(got.imag) and np.array_equal(got, got.T)
    if precision == "fp64":
        assert err <= 1e-10
        return
    pred = pr.normwise_error(predicted((name, "slice-real"), [synth.pack_real_pairs(m) for m in mr],
                                       _factors(name, True), sl.weights_q(), precision, sl.n_s, plan).real, ref)
    rho = np.abs(np.linalg.eigvalsh(ref.real)).max()
    eig = pr.normalised_eig_error(got, ref, rho)
    print(f"[full-shape] emulated {pred:.3e}, ratio {err / pred:.2f}, eigenvalue error {eig:.3e} Ha", flush=True)
    assert err <= 4.0 * pred + 1e-12, (name, precision, cfg_id, err, pred)
    assert eig <= 1e-6


@pytest.mark.parametrize("precision", ["fp64", "bf16x3"])
def test_eibz_sum_at_si_like_shapes(precision):
    """The EIBZ-restricted q sum of the Si-like workload (154 of its 512 pairs, weights
    w_q / N_{k,q} for its 8 irreducible k) against the oracle's restricted sum."""
    import paper_1003_0524_amd as lib
    from paper_1003_0524_amd import symmetry as sy
    cfg = synth.make_config("c2")
    ops = sy.point_group(cfg.lattice)
    k_idx, _ = sy.irreducible(cfg.q_frac, ops)
    w_kq = np.stack([sy.eibz_weights(cfg.q_frac[i], cfg.q_frac, ops, cfg.weights_q())[0] for i in k_idx])
    E, D, C = synth.coulomb_blocks(cfg)
    print(f"[full-shape] c2 EIBZ {precision}: {np.count_nonzero(w_kq)} pairs", flush=True)
    ex = lib.Exchange(cfg.n_bands, cfg.n_pw, cfg.ch_nrad, cfg.n_occ, E, D, C, w_q=cfg.weights_q(),
                      precision=precision, form="herk", batched=True, w_kq=w_kq)
    Ms = [torch.from_numpy(np.concatenate([synth.m_block(cfg, k, q).ravel() for q in range(cfg.n_q)
                                           if w_kq[k, q] != 0])).cuda() for k in range(cfg.n_k)]
    Vs = [V.cpu().numpy() for V in ex.matrix_all(Ms)]
    plan = ex.accumulation_plan()
    ex.close()
    v = [vx.assemble_v(E[q], D, C) for q in range(cfg.n_q)]
    L = [chol.cholesky(a) for a in v] if precision != "fp64" else None
    for k in range(cfg.n_k):
        keep = [q for q in range(cfg.n_q) if w_kq[k, q] != 0]
        blocks = [synth.m_block(cfg, k, q) for q in keep]
        ref = vx.vx_k(blocks, [v[q] for q in keep], w_kq[k, keep])
        err = pr.normwise_error(Vs[k], ref)
        if precision == "fp64":
            assert err <= 1e-10, (k, err)
        else:
            pred = pr.normwise_error(pr.vx_k_emulated(blocks, [L[q] for q in keep], w_kq[k, keep], precision,
                                                      cfg.n_s, plan), ref)
            assert err <= 4.0 * pred + 1e-12, (k, err, pred)


def test_si_like_full_mesh_bf16x3():
    """The Si-like workload whole (8 irreducible k x 64 q, complex128 M), as the benchmark
    runs it in bf16x3: within 4x the predicted error and <= 1e-6 Ha on the normalised
    eigenvalues of every k."""
    import paper_1003_0524_amd as lib
    cfg = synth.make_config("c2")
    E, D, C = synth.coulomb_blocks(cfg)
    print("[full-shape] c2 full mesh bf16x3", flush=True)
    ex = lib.Exchange(cfg.n_bands, cfg.n_pw, cfg.ch_nrad, cfg.n_occ, E, D, C, w_q=cfg.weights_q(),
                      precision="bf16x3", form="herk", batched=True)
    Vs = [V.cpu().numpy() for V in ex.matrix_all([torch.from_numpy(synth.m_all(cfg, k)).cuda()
                                                  for k in range(cfg.n_k)])]
    plan = ex.accumulation_plan()
    ex.close()
    v = [vx.assemble_v(E[q], D, C) for q in range(cfg.n_q)]
    L = [chol.cholesky(a) for a in v]
    refs = [vx.vx_k([synth.m_block(cfg, k, q) for q in range(cfg.n_q)], v, cfg.weights_q())
            for k in range(cfg.n_k)]
    rho = max(np.abs(np.linalg.eigvalsh(vx.hermitian_part(r))).max() for r in refs)
    for k in range(cfg.n_k):
        blocks = [synth.m_block(cfg, k, q) for q in range(cfg.n_q)]
        err = pr.normwise_error(Vs[k], refs[k])
        pred = pr.normwise_error(pr.vx_k_emulated(blocks, L, cfg.weights_q(), "bf16x3", cfg.n_s, plan), refs[k])
        eig = pr.normalised_eig_error(Vs[k], refs[k], rho)
        print(f"[full-shape] c2 k={k}: error {err:.3e}, predicted {pred:.3e}, eigenvalues {eig:.3e} Ha", flush=True)
        assert err <= 4.0 * pred + 1e-12, (k, err, pred)
        assert eig <= 1e-6, (k, eig)
