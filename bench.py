#!/usr/bin/env python3
"""Benchmark of the nonlocal exchange matrix V^x on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c2] [--no-cpu]

One step = one outer-iteration evaluation on the workload: V^x(k) for every
irreducible k (all q, all occupied n'') through exchange_matrix_all, followed
by the exchange energy E_x = 1/2 sum_k w_k Tr(rho_k V_k) (exchange_energy_device:
the energy stays in device memory, as in a loop that keeps its results on the
GPU; it is read back once after the timed steps and checked against the
synchronising exchange_energy).
The Coulomb matrix preparation (FP64 Cholesky, once per self-consistency
cycle) happens before the timed region and is reported as init_ms.

Forms measured on the same resident inputs:
  * plain     -- FP64, GEMM form (W = v A then A^H W), one launch per (k,q), no graph;
  * fp64      -- FP64 Cholesky/HERK form, one persistent launch in a HIP graph;
  * fp32, bf16x3, bf16x6 -- the same batched form with reduced-precision products.
The headline ("value") is the fastest batched mixed-precision mode whose
eigenvalue error against the FP64 oracle, normalised to a 1 Ha spectral radius,
is <= 1e-6 Ha. Prints one JSON line.

Also timed, outside the step (it is computed once per self-consistency cycle):
the Gamma-point term's lattice sum (exchange_gamma_term, beta = 0.005, on the
workload's q mesh), reported under "gamma_term".
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "V^x GFLOP/s & k-points/s: batched mixed-prec vs plain FP64, ≤1e-6 Ha error"
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2516.6, "bf16x6": 2516.6}
DTYPE = {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16", "bf16x6": "bf16"}
HBM_PEAK_GBS = 8000.0
WORKLOADS = {
    "c2": "Si-like fcc cell, 4x4x4 Gamma-centred q mesh (64 q), 8 irreducible k, "
          "N_MB=620 (260 plane waves + 360 MT: 2 atoms, n_rad(l)=10-l, l<=4), 24 bands, 4 occupied, "
          "M complex128",
    "c1": "1 k, 8 random non-Gamma q, N_MB=300 (150 PW + 150 MT), 16 bands, 8 occupied",
}


def _kernel_src_hash() -> str:
    h = hashlib.sha256()
    for f in ("tile.hpp", "fused.hpp", "common.hpp", "aux.hpp", "exchange.hip"):
        with open(os.path.join(ROOT, "paper_1003_0524_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _traffic(workload: str, mode: str, kernel_cfg: int = -1):
    """HBM bytes per launch of the dominant kernel from committed rocprofv3 counters,
    or None when they were taken on a different kernel source."""
    p = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    e = d.get(mode)
    if e and "src_hash" not in e:        # one record per configuration id
        e = e.get(str(kernel_cfg))
    if not e or e.get("src_hash") != _kernel_src_hash():
        return None
    if e.get("cfg_id") is not None and e.get("cfg_id") != kernel_cfg:
        return None                      # counters of another configuration
    return e.get("bytes_per_launch")


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--modes", default="fp32,bf16x3,bf16x6")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-gamma", action="store_true", help="skip timing the Gamma-point lattice sum")
    ap.add_argument("--no-inversion", action="store_true", help="skip the inversion-symmetric variant")
    ap.add_argument("--no-eibz", action="store_true", help="skip the EIBZ-restricted q sum")
    ap.add_argument("--no-backx", action="store_true", help="skip timing the back-transform to the LAPW basis")
    ap.add_argument("--only", default=None, help="run a single batched mode (profiling runs)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device-to-device 3 times (scales HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the exchange path here is built and timed on a "
              "single MI355X (sharding the q sum over GPUs, with one all-reduce of the FP64 partial V, is not run).",
              file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_1003_0524_amd as lib
    import synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    dev = torch.device("cuda:0")
    if args.calibrate_copy:
        n = args.calibrate_copy * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes_read": n * 4, "bytes_written": n * 4, "copies": 3}))
        return 0
    cfg = synth.make_config(args.workload)
    E, D, C = synth.coulomb_blocks(cfg)
    mdt = np.complex128
    Ms = [torch.from_numpy(synth.m_all(cfg, k, mdt)).to(dev) for k in range(cfg.n_k)]
    torch.cuda.synchronize()
    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    log(f"[bench] workload {args.workload}: n_k={cfg.n_k} n_q={cfg.n_q} N_MB={cfg.n_mb(0)} "
        f"n_b={cfg.n_bands[0]} n_occ={cfg.n_occ}")

    def make(precision, form, batched, inversion=False, w_kq=None):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        blocks = synth.coulomb_blocks_real(cfg) if inversion else (E, D, C)
        ex = lib.Exchange(cfg.n_bands, cfg.n_pw, cfg.ch_nrad, cfg.n_occ, *blocks,
                          w_q=cfg.weights_q(), precision=precision, form=form, batched=batched,
                          inversion=inversion, w_kq=w_kq)
        torch.cuda.synchronize()
        return ex, (time.perf_counter() - t0) * 1e3

    outs = [torch.empty(nb * nb, dtype=torch.complex128, device=dev) for nb in cfg.n_bands]
    e_dev = torch.zeros(1, dtype=torch.float64, device=dev)

    def step(ex, m_in):
        # V(k) for every k and E_x, both left in device memory: no host round trip per step
        ex.matrix_all(m_in, outs)
        ex.energy_device(e_dev)

    def timed(ex, steps, warmup, kernel_timing=False, m_in=None):
        m_in = Ms if m_in is None else m_in
        if kernel_timing:
            ex.timing(steps)          # re-captures the graph: before the warm-up
        for _ in range(max(1, warmup)):
            step(ex, m_in)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            step(ex, m_in)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        energy = float(e_dev.item())
        e_host = ex.energy()                      # the synchronising entry point agrees
        if abs(energy - e_host) > 1e-12 * max(1.0, abs(e_host)):
            raise RuntimeError(f"device energy {energy} != host energy {e_host}")
        kt = ex.kernel_ms() if kernel_timing else None
        return ms, energy, kt

    # the q-mesh divisions (a Gamma-centred mesh has n_i distinct fractions on axis i)
    mesh = tuple(len(np.unique(np.round(cfg.q_frac[:, i], 12))) for i in range(3))
    if int(np.prod(mesh)) != cfg.n_q:
        mesh = None
    gamma = None
    btx = None

    results = {}
    modes = [args.only] if args.only else ["plain", "fp64"] + [m for m in args.modes.split(",") if m]
    for mode in modes:
        if mode == "plain":
            ex, init_ms = make("fp64", "gemm", False)
            steps, warm = max(3, args.steps // 10), max(1, args.warmup // 5)
        else:
            ex, init_ms = make(mode, "herk", True)
            steps, warm = args.steps, args.warmup
        log(f"[bench] {mode}: init {init_ms:.1f} ms, timing {steps} steps")
        ms, energy, kt = timed(ex, steps, warm, kernel_timing=(mode != "plain"))
        V = [o.view(nb, nb).T.cpu().numpy() for o, nb in zip(outs, cfg.n_bands)]
        results[mode] = dict(ms=ms, init_ms=init_ms, energy=energy, kt=kt, V=V,
                             flops_nom=ex.query(1), flops_exec=ex.query(2), bytes_alg=ex.query(4),
                             items=int(ex.query(0)), cfg=int(ex.query(3)), tuned=int(ex.query(8)),
                             ws_bytes=ex.query(9), fused=bool(ex.query(10)))
        log(f"[bench] {mode}: {ms:.4f} ms/step, E_x = {energy:.8f}"
            + (f", main kernel {kt[0]:.4f} ms, sparse kernel {kt[1]:.4f} ms" if kt else "")
            + f", config {results[mode]['cfg']}{' (autotuned)' if results[mode]['tuned'] else ''}")
        if gamma is None and mesh is not None and not args.no_gamma:
            # Gamma-point term (computed once per self-consistency cycle): lattice-sum kernel, HIP events
            c_gamma = ex.gamma_term(cfg.recip(), mesh, 0.005, apply=False)
            kms = []
            for _ in range(5):
                ex.gamma_term(cfg.recip(), mesh, 0.005, apply=False)
                kms.append(ex.gamma_kernel_ms()[0])
            n_terms = ex.gamma_kernel_ms()[1]
            gamma = {"C": c_gamma, "beta": 0.005, "mesh": list(mesh), "terms": n_terms,
                     "kernel_ms": round(float(np.mean(kms)), 5),
                     "terms_per_s": round(n_terms / (float(np.mean(kms)) * 1e-3), 1)}
            log(f"[bench] gamma term: C = {c_gamma:.12f}, {n_terms} terms, lattice-sum kernel {gamma['kernel_ms']:.4f} ms")
        if btx is None and mode == "fp64" and not args.no_backx:
            # back-transform of V(k=0) to an LAPW basis of n_G functions (synthetic Z = S c)
            btx = []
            rng = np.random.default_rng(20)
            for nG in (400, 2000):
                nb0 = cfg.n_bands[0]
                Zh = rng.standard_normal((nG, nb0)) + 1j * rng.standard_normal((nG, nb0))
                Zd = torch.from_numpy(np.ascontiguousarray(Zh.T)).to(dev).T
                VG = torch.empty(nG * nG, dtype=torch.complex128, device=dev)
                ex.back_transform(0, Zd, VG)
                kms = []
                for _ in range(5):
                    ex.back_transform(0, Zd, VG)
                    kms.append(ex.query(13))
                t_k = float(np.mean(kms))
                fl, by = 8.0 * nG * nG * nb0, 16.0 * nG * nG + 2 * 16.0 * nG * nb0
                ridge = PEAK_TFLOPS["fp64"] * 1e12 / (HBM_PEAK_GBS * 1e9)
                bound = "mfma" if fl / by >= ridge else "hbm"
                frac = (fl / (t_k * 1e-3) / 1e12 / PEAK_TFLOPS["fp64"] if bound == "mfma"
                        else by / (t_k * 1e-3) / 1e9 / HBM_PEAK_GBS)
                btx.append({"n_G": nG, "n_b": nb0, "kernel_ms": round(t_k, 5), "bound": bound,
                            "tflops": round(fl / (t_k * 1e-3) / 1e12, 3),
                            "gbps": round(by / (t_k * 1e-3) / 1e9, 1), "frac": round(frac, 4)})
                log(f"[bench] back-transform n_G={nG}: product kernel {t_k:.4f} ms, "
                    f"{btx[-1]['tflops']} TFLOP/s, {btx[-1]['gbps']} GB/s ({bound}-bound, {frac:.2%})")
        ex.close()

    # errors against the float64 oracle (all k)
    from oracle import precision as pr
    from oracle import vx
    v = [vx.assemble_v(E[q], D, C) for q in range(cfg.n_q)]
    refs = [vx.vx_k([synth.m_block(cfg, k, q) for q in range(cfg.n_q)], v, cfg.weights_q())
            for k in range(cfg.n_k)]
    rho = max(np.abs(np.linalg.eigvalsh(vx.hermitian_part(r))).max() for r in refs)
    for mode, r in results.items():
        r["err_norm"] = max(pr.normwise_error(a, b) for a, b in zip(r["V"], refs))
        r["err_eig_ha"] = max(pr.normalised_eig_error(a, b, rho) for a, b in zip(r["V"], refs))
        log(f"[bench] {mode}: normwise {r['err_norm']:.3e}, eigenvalue error {r['err_eig_ha']:.3e} Ha (normalised)")

    mixed = [m for m in results if m not in ("plain", "fp64") and results[m]["err_eig_ha"] <= 1e-6]
    head = min(mixed, key=lambda m: results[m]["ms"]) if mixed else ("fp64" if "fp64" in results else modes[0])
    H = results[head]
    value = H["flops_nom"] / (H["ms"] * 1e-3) / 1e9

    # inversion-symmetric variant (real v and real projections, bands packed in pairs) in the
    # headline's precision on the same workload shapes
    inv = None
    if not args.no_inversion and head not in ("plain",):
        Mr = [torch.from_numpy(synth.m_all_real_packed(cfg, k, mdt)).to(dev) for k in range(cfg.n_k)]
        exr, init_r = make(head, "herk", True, inversion=True)
        ms_r, e_r, kt_r = timed(exr, args.steps, args.warmup, kernel_timing=True, m_in=Mr)
        Vr = [o.view(nb, nb).T.cpu().numpy() for o, nb in zip(outs, cfg.n_bands)]
        nom_r, cfg_r = exr.query(1), int(exr.query(3))
        exr.close()
        Er, Dr, Cr = synth.coulomb_blocks_real(cfg)
        vr = [vx.assemble_v(Er[q], Dr, Cr) for q in range(cfg.n_q)]
        refs_r = [vx.vx_k([synth.m_block_real(cfg, k, q) for q in range(cfg.n_q)], vr, cfg.weights_q())
                  for k in range(cfg.n_k)]
        rho_r = max(np.abs(np.linalg.eigvalsh(r.real)).max() for r in refs_r)
        inv = {"mode": head, "ms_per_step": round(ms_r, 5), "main_kernel_ms": round(kt_r[0], 5),
               "gflops_nominal_real": round(nom_r / (ms_r * 1e-3) / 1e9, 3),
               "kpoints_per_s": round(cfg.n_k / (ms_r * 1e-3), 1),
               "speedup_vs_complex": round(H["ms"] / ms_r, 3), "config": cfg_r,
               "err_normwise": max(pr.normwise_error(a, b) for a, b in zip(Vr, refs_r)),
               "err_eig_ha": max(pr.normalised_eig_error(a, b, rho_r) for a, b in zip(Vr, refs_r))}
        log(f"[bench] inversion variant ({head}): {ms_r:.4f} ms/step, main kernel {kt_r[0]:.4f} ms, "
            f"{H['ms'] / ms_r:.2f}x the complex step, eigenvalue error {inv['err_eig_ha']:.3e} Ha")

    # q sum restricted to the extended irreducible wedge EIBZ(k) of each irreducible k (the
    # workload's k are the irreducible points of its mesh), weights w_q / N_{k,q}
    eibz = None
    if not args.no_eibz and mesh is not None and head not in ("plain",):
        from paper_1003_0524_amd import symmetry as sy
        ops = sy.point_group(cfg.lattice)
        k_idx, _ = sy.irreducible(cfg.q_frac, ops)
        if len(k_idx) == cfg.n_k:
            w_kq = np.stack([sy.eibz_weights(cfg.q_frac[i], cfg.q_frac, ops, cfg.weights_q())[0] for i in k_idx])
            Me = [torch.from_numpy(np.concatenate([synth.m_block(cfg, k, q, mdt).ravel()
                                                   for q in range(cfg.n_q) if w_kq[k, q] != 0])).to(dev)
                  for k in range(cfg.n_k)]
            exe, _ = make(head, "herk", True, w_kq=w_kq)
            ms_e, _, kt_e = timed(exe, args.steps, args.warmup, kernel_timing=True, m_in=Me)
            Ve = [o.view(nb, nb).T.cpu().numpy() for o, nb in zip(outs, cfg.n_bands)]
            cfg_e, fused_e, split_e = int(exe.query(3)), bool(exe.query(10)), int(exe.query(14))
            exe.close()
            refs_e = []
            for k in range(cfg.n_k):
                keep = [q for q in range(cfg.n_q) if w_kq[k, q] != 0]
                refs_e.append(vx.vx_k([synth.m_block(cfg, k, q) for q in keep], [v[q] for q in keep], w_kq[k, keep]))
            n_pairs = int(np.count_nonzero(w_kq))
            eibz = {"mode": head, "pairs": n_pairs, "pairs_full_mesh": cfg.n_k * cfg.n_q,
                    "ms_per_step": round(ms_e, 5), "main_kernel_ms": round(kt_e[0], 5),
                    "sparse_kernel_ms": round(kt_e[1], 5), "config": cfg_e, "fused": fused_e,
                    "items_per_band_chunk": split_e,
                    "kpoints_per_s": round(cfg.n_k / (ms_e * 1e-3), 1),
                    "speedup_vs_full_mesh": round(H["ms"] / ms_e, 3),
                    "err_normwise": max(pr.normwise_error(a, b) for a, b in zip(Ve, refs_e))}
            log(f"[bench] EIBZ q sum ({head}): {n_pairs} of {cfg.n_k * cfg.n_q} pairs, {ms_e:.4f} ms/step, "
                f"main kernel {kt_e[0]:.4f} ms, {H['ms'] / ms_e:.2f}x the full-mesh step, config {cfg_e}"
                f"{' (an item per band chunk)' if split_e else ''}")

    # roofline of the dominant kernel, timed live with graph event nodes. Its bound
    # follows from its arithmetic intensity (algorithmic flops / algorithmic HBM
    # bytes) against the ridge point peak_flops / peak_bandwidth of its dtype.
    roof = None
    if H["kt"] and H["kt"][0] > 0:
        t_main, t_sparse = H["kt"][0], H["kt"][1]
        m_bytes = sum(cfg.n_occ * cfg.n_bands[k] * cfg.n_mb(q) for k in range(cfg.n_k) for q in range(cfg.n_q)) * 16.0
        if H["fused"]:
            name, t_k = "fused_kernel (block-sparse rows, dense rows on MFMA, band contraction; M read once)", t_main
            flops, byts = H["flops_exec"], H["bytes_alg"]
        elif t_main >= t_sparse:
            name, t_k = "tile_kernel (dense rows Y = L^H A on MFMA + band contraction)", t_main
            flops, byts = H["flops_exec"], H["ws_bytes"] + (H["bytes_alg"] - m_bytes)
        else:
            name, t_k = "sparse_kernel (block-sparse rows, packs the tile kernel's operands)", t_sparse
            flops, byts = 0.0, m_bytes + H["ws_bytes"]
        peak_f = PEAK_TFLOPS[head]
        ridge = peak_f * 1e12 / (HBM_PEAK_GBS * 1e9)
        intensity = flops / byts if byts > 0 else float("inf")
        if intensity < ridge:
            ach = byts / (t_k * 1e-3) / 1e9
            roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(ach / HBM_PEAK_GBS, 5)}
        else:
            ach = flops / (t_k * 1e-3) / 1e12
            roof = {"bound": "mfma", "achieved": round(ach, 3), "peak": peak_f, "unit": "TFLOP/s",
                    "frac": round(ach / peak_f, 5)}
        roof.update({"traffic": _traffic(args.workload, head, H["cfg"]), "kernel": name, "kernel_ms": round(t_k, 5),
                     "launches_timed": H["kt"][2], "algorithmic_bytes_per_launch": byts,
                     "algorithmic_flops_per_launch": flops,
                     "intensity_flop_per_byte": round(intensity, 2), "ridge_flop_per_byte": round(ridge, 1),
                     "mfma_frac": round(flops / (t_k * 1e-3) / 1e12 / peak_f, 5)})

    # CPU baseline: the oracle as it stands on the host cores, bounded sample
    cpu = None
    if not args.no_cpu:
        try:
            from threadpoolctl import threadpool_info
            threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
        except Exception:
            threads = os.cpu_count()
        mb = [[synth.m_block(cfg, k, q) for q in range(cfg.n_q)] for k in range(cfg.n_k)]
        reps, t_cpu = 0, 0.0
        t0 = time.perf_counter()
        while t_cpu < 10.0 and reps < 50:
            for k in range(cfg.n_k):
                vx.vx_k(mb[k], v, cfg.weights_q())
            reps += 1
            t_cpu = time.perf_counter() - t0
        fl = H["flops_nom"] * reps
        cpu = {"value": round(fl / t_cpu / 1e9, 3), "unit": "GFLOP/s", "cores": threads, "kind": "oracle",
               "sample": f"{reps} full evaluation(s) of all {cfg.n_k} k x {cfg.n_q} q with the dense-v "
                         f"NumPy oracle ({t_cpu:.1f} s); GFLOP counted as the method's nominal flops",
               "ms_per_step": round(t_cpu / reps * 1e3, 2)}

    sparse = None
    if H["kt"] and H["kt"][1] > 0 and not H["fused"]:
        # block-sparse rows: read the MT rows of M (+ multipole rows), write Y_s
        n_s, n_ch = cfg.n_s, cfg.n_ch
        elems = sum(cfg.n_occ * cfg.n_bands[k] for k in range(cfg.n_k)) * cfg.n_q
        msz = 16 if mdt == np.complex128 else 8
        ysz = 16 if head == "fp64" else 8
        byts = elems * ((n_s + n_ch) * msz + n_s * ysz)
        sparse = {"kernel": "sparse_kernel", "kernel_ms": round(H["kt"][1], 5),
                  "algorithmic_GBps": round(byts / (H["kt"][1] * 1e-3) / 1e9, 1),
                  "frac_hbm": round(byts / (H["kt"][1] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}

    P = results.get("plain")
    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "GFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(H["ms"], 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPE[head], "data": "synthetic (seeded SplitMix64/Box-Muller M, synthetic PD Coulomb blocks)",
        "config": {"workload": f"{args.workload}: {WORKLOADS[args.workload]}", "mode": head,
                   "form": "cholesky-herk, one persistent launch in a HIP graph",
                   "kernel_config": H["cfg"], "autotuned": H["tuned"]},
        "kpoints_per_s": round(cfg.n_k / (H["ms"] * 1e-3), 1),
        "pairs_per_s": round(cfg.n_k * cfg.n_q / (H["ms"] * 1e-3), 1),
        "gflops_executed": round(H["flops_exec"] / (H["ms"] * 1e-3) / 1e9, 3),
        "err_eig_ha": H["err_eig_ha"], "err_normwise": H["err_norm"],
        "init_ms": round(H["init_ms"], 2),
        "roofline": roof, "cpu_baseline": cpu, "sparse_rows": sparse, "gamma_term": gamma,
        "inversion_variant": inv, "eibz_q_sum": eibz, "back_transform": btx,
        "modes": {m: {"ms_per_step": round(r["ms"], 5),
                      "gflops": round(r["flops_nom"] / (r["ms"] * 1e-3) / 1e9, 3),
                      "err_eig_ha": r["err_eig_ha"], "err_normwise": r["err_norm"],
                      "main_kernel_ms": (round(r["kt"][0], 5) if r["kt"] else None),
                      "config": r["cfg"], "fused": r["fused"], "tuned": r["tuned"]}
                  for m, r in results.items()},
        "speedup_vs_plain_fp64": (round(P["ms"] / H["ms"], 2) if P else None),
    }
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
