#!/usr/bin/env python3
"""Benchmark of the nonlocal exchange matrix V^x on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c4] [--also c3,c2] [--no-cpu]

One step = one outer-iteration evaluation of a workload: V^x(k) for every
irreducible k (all q, all occupied n''), followed by the exchange energy
E_x = 1/2 sum_k w_k Tr(rho_k V_k) left in device memory (exchange_energy_device;
read back once after the timed steps and checked against exchange_energy).
The Coulomb matrix preparation (FP64 Cholesky, once per self-consistency cycle)
happens before the timed region and is reported as init_ms.

The headline workload is the SrTiO3-like one (c4: 20 k x 216 q, N_MB 2000-2600,
100 bands, 20 occupied), the largest that fits one GPU; the ZnO-like one (c3) and
the Si-like one (c2, with the widening rows: inversion-symmetric variant, EIBZ q
sum, Gamma-point term, back-transform) are reported in the same line.

Forms measured on each workload:
  * plain  -- FP64 GEMM form (W = v A, then A^H W), one launch of each kernel per (k,q), no graph;
  * fp64   -- FP64 Cholesky/HERK form, batched (one launch over all (k,q) in a HIP graph, or
              over the q of one k where M is streamed per k);
  * fp32, bf16x3, bf16x6 -- the batched HERK form with reduced-precision products, one
              persistent launch over all (k,q) replayed from a HIP graph.
M is drawn on the GPU by the seeded device generator (synth/csrc/synth.hip): complex64 and
resident for the reduced-precision forms of c3 and c4 (29 / 159 GB), complex128 for the FP64
forms -- resident on c2, drawn per k outside the timed region on c3 and c4 (58 / 318 GB would
not fit), where the step time is the sum of the per-k times.
The headline ("value") is the fastest reduced-precision mode whose eigenvalue error, normalised
to a 1 Ha spectral radius, is <= 1e-6 Ha against the float64 oracle (c2: every k computed here;
c3 / c4: the oracle's V(k = 0) over all q, stored in tests/golden by make_vx_golden.py).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

# Kernel arguments in device memory (a HIP runtime setting, read when HIP starts): each kernel of a
# step then starts without reading its arguments from host memory; the Si-like step is 3-5 us
# shorter with it. A value already in the environment is kept.
os.environ.setdefault("HIP_FORCE_DEV_KERNARG", "1")

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "V^x GFLOP/s & k-points/s: batched mixed-prec vs plain FP64, ≤1e-6 Ha error"
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2516.6, "bf16x6": 2516.6}
DTYPE = {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16", "bf16x6": "bf16", "plain": "f64"}
HBM_PEAK_GBS = 8000.0
MIXED = ("fp32", "bf16x3", "bf16x6")
# the FP64 forms are timed over fewer steps when the requested count would take longer than this
SLOW_FORM_BUDGET_S = 20.0
WORKLOADS = {
    "c4": "SrTiO3-like simple cubic cell (a = 7.38 bohr), 6x6x6 Gamma-centred q mesh (216 q), 20 irreducible k, "
          "N_MB(q) uniform in [2000, 2600] (1200 multipole-free MT functions in 180 (atom, L, M) channels of "
          "5 atoms, l <= 5, + 180 multipole functions + 622-1220 plane waves), 100 bands, 20 occupied",
    "c3": "ZnO-like hexagonal cell (a = 6.14, c = 9.84 bohr), 6x6x4 Gamma-centred q mesh (144 q), 21 irreducible k, "
          "N_MB(q) uniform in [820, 1400] (455 multipole-free MT functions in 100 channels of 4 atoms, l <= 4, "
          "+ 100 multipole functions + 272-844 plane waves), 60 bands, 18 occupied",
    "c2": "Si-like fcc cell (a = 10.26 bohr), 4x4x4 Gamma-centred q mesh (64 q), 8 irreducible k, "
          "N_MB = 620 (260 plane waves + 360 MT: 2 atoms, n_rad(l) = 10 - l, l <= 4), 24 bands, 4 occupied",
    "c1": "1 k, 8 random non-Gamma q, N_MB = 300 (150 plane waves + 150 MT), 16 bands, 8 occupied",
}
# workloads whose complex128 M does not stay resident: the FP64 forms take it per k
STREAMED = ("c3", "c4")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _kernel_file(kernel_cfg: int) -> str:
    """The source file that defines the main kernel of a configuration id."""
    if 180 <= kernel_cfg < 200:
        return "wide.hpp"
    if kernel_cfg >= 100:
        return "fused.hpp"
    return "tile.hpp"


def _kernel_src_hash(kernel_cfg: int) -> str:
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_1003_0524_amd", "csrc", _kernel_file(kernel_cfg)), "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()[:16]


def _traffic(workload: str, mode: str, kernel_cfg: int = -1):
    """HBM bytes per launch of the dominant kernel from committed rocprofv3 counters,
    or None when they were taken on a different kernel source or configuration."""
    p = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    e = d.get(mode)
    if e and "src_hash" not in e:        # one record per configuration id
        e = e.get(str(kernel_cfg))
    if not e or e.get("src_hash") != _kernel_src_hash(int(e.get("cfg_id", kernel_cfg))):
        return None
    if e.get("cfg_id") is not None and e.get("cfg_id") != kernel_cfg:
        return None
    return e.get("bytes_per_launch")


def nominal_flops_pair(cfg, k, q):
    """The method's flops for one (k, q) pair: sparse-aware, complex multiply-add = 8,
    Hermitian upper triangle of the band contraction (the library's accounting)."""
    nb, nocc = cfg.n_bands[k], cfg.n_occ
    R = nocc * nb
    nd = cfg.n_d(q)
    sp = sum(8.0 * (b - 1) ** 2 * R for b in cfg.ch_nrad)
    return 8.0 * nd * nd * R + sp + 16.0 * cfg.n_s * R + 4.0 * nb * (nb + 1.0) * cfg.n_mb(q) * nocc


class Bench:
    def __init__(self, args, torch, lib, synth):
        self.args, self.torch, self.lib, self.synth = args, torch, lib, synth
        self.dev = torch.device("cuda:0")

    # ------------------------------------------------------------------
    def setup(self, name):
        import numpy as np
        synth = self.synth
        t0 = time.perf_counter()
        self.name = name
        self.cfg = cfg = synth.make_config(name)
        self.E, self.D, self.C = synth.coulomb_blocks(cfg)
        self.E_dev = [self.torch.from_numpy(e).to(self.dev) for e in self.E]
        self.outs = [self.torch.empty(nb * nb, dtype=self.torch.complex128, device=self.dev) for nb in cfg.n_bands]
        self.e_dev = self.torch.zeros(1, dtype=self.torch.float64, device=self.dev)
        self.streamed = name in STREAMED
        self.mdt_mixed = "c64" if self.streamed else "c128"
        self.golden = None
        self.copy_gbs = None
        self.measure_copy()
        if self.streamed:
            g = {}
            for dt in ("c64", "c128"):
                p = os.path.join(ROOT, "tests", "golden", f"vx_{name}_k0_{dt}.npy")
                g[dt] = np.load(p) if os.path.exists(p) else None
            self.golden = g
        log(f"[bench] {name}: n_k={cfg.n_k} n_q={cfg.n_q} N_MB={min(cfg.n_mb(q) for q in range(cfg.n_q))}.."
            f"{max(cfg.n_mb(q) for q in range(cfg.n_q))} n_b={cfg.n_bands[0]} n_occ={cfg.n_occ}, "
            f"host inputs {time.perf_counter() - t0:.1f} s")

    def make(self, precision, form, batched, inversion=False, w_kq=None):
        torch, cfg = self.torch, self.cfg
        # the Coulomb blocks are handed over in device memory, as the workload's other inputs are
        if inversion:
            Er, Dr, Cr = self.synth.coulomb_blocks_real(cfg)
            blocks = ([torch.from_numpy(e).to(self.dev) for e in Er], Dr, Cr)
        else:
            blocks = (self.E_dev, self.D, self.C)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ex = self.lib.Exchange(cfg.n_bands, cfg.n_pw, cfg.ch_nrad, cfg.n_occ, *blocks, w_q=cfg.weights_q(),
                               precision=precision, form=form, batched=batched, inversion=inversion, w_kq=w_kq)
        torch.cuda.synchronize()
        return ex, (time.perf_counter() - t0) * 1e3

    def resident_m(self, dtype):
        return [self.synth.m_all_device(self.cfg, k, dtype, self.dev) for k in range(self.cfg.n_k)]

    def v_host(self):
        return [o.view(nb, nb).T.cpu().numpy() for o, nb in zip(self.outs, self.cfg.n_bands)]

    # one step on resident inputs: V(k) for every k and E_x, both left in device memory
    def timed(self, ex, steps, warmup, m_in, kernel_timing=False, budget_s=None):
        """Mean ms per step over `steps` steps after `warmup` untimed ones. With `budget_s`, a form whose
        warm-up step shows that `steps` steps would take longer is timed over fewer (at least 3); the
        count used is left in `self.last_steps`."""
        torch = self.torch
        for w in range(max(1, warmup)):
            t0 = time.perf_counter()
            ex.matrix_all(m_in, self.outs)
            ex.energy_device(self.e_dev)
            torch.cuda.synchronize()
            t_warm = time.perf_counter() - t0
        if budget_s is not None and t_warm * steps > budget_s:
            steps = max(3, int(budget_s / t_warm))
        self.last_steps = steps
        if kernel_timing:
            ex.timing(steps)          # re-captures the graph: one more untimed step after it
            ex.matrix_all(m_in, self.outs)
            ex.energy_device(self.e_dev)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            ex.matrix_all(m_in, self.outs)
            ex.energy_device(self.e_dev)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        energy = float(self.e_dev.item())
        e_host = ex.energy()
        if abs(energy - e_host) > 1e-12 * max(1.0, abs(e_host)):
            raise RuntimeError(f"device energy {energy} != host energy {e_host}")
        return ms, energy, (ex.kernel_ms() if kernel_timing else None)

    # one step with M drawn per k outside the timed region: the sum of the per-k times
    def timed_streamed(self, ex, dtype="c128"):
        torch, cfg, synth = self.torch, self.cfg, self.synth
        n_max = max(cfg.m_elems(k) for k in range(cfg.n_k))
        buf = torch.empty(n_max, dtype=torch.complex128 if dtype == "c128" else torch.complex64, device=self.dev)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        # warm-up: the first call sizes the context's workspaces
        m0 = synth.m_all_device(cfg, 0, dtype, self.dev, out=buf[:cfg.m_elems(0)])
        ex.matrix(0, m0, self.outs[0])
        torch.cuda.synchronize()
        total = 0.0
        per_k = []
        for k in range(cfg.n_k):
            mk = synth.m_all_device(cfg, k, dtype, self.dev, out=buf[:cfg.m_elems(k)])
            torch.cuda.synchronize()
            e0.record()
            ex.matrix(k, mk, self.outs[k])
            e1.record()
            torch.cuda.synchronize()
            per_k.append(e0.elapsed_time(e1))
            total += per_k[-1]
        e0.record()
        ex.energy_device(self.e_dev)
        e1.record()
        torch.cuda.synchronize()
        total += e0.elapsed_time(e1)
        energy = float(self.e_dev.item())
        del buf
        return total, energy, per_k

    # ------------------------------------------------------------------
    def errors(self, V, ref_kind):
        """(normwise, normalised eigenvalue error) against the oracle: every k (c1/c2) or
        the stored V(k = 0) of the whole q sum (c3/c4)."""
        from oracle import precision as pr
        if self.streamed:
            ref = self.golden.get(ref_kind)
            if ref is None:
                return None, None
            import numpy as np
            rho = float(np.abs(np.linalg.eigvalsh(0.5 * (ref + ref.conj().T))).max())
            return pr.normwise_error(V[0], ref), pr.normalised_eig_error(V[0], ref, rho)
        refs, rho = self.oracle_refs()
        return (max(pr.normwise_error(a, b) for a, b in zip(V, refs)),
                max(pr.normalised_eig_error(a, b, rho) for a, b in zip(V, refs)))

    def oracle_refs(self):
        if getattr(self, "_refs", None) is None:
            import numpy as np
            from oracle import vx
            cfg = self.cfg
            v = [vx.assemble_v(self.E[q], self.D, self.C) for q in range(cfg.n_q)]
            refs = [vx.vx_k([self.synth.m_block(cfg, k, q) for q in range(cfg.n_q)], v, cfg.weights_q())
                    for k in range(cfg.n_k)]
            rho = max(np.abs(np.linalg.eigvalsh(vx.hermitian_part(r))).max() for r in refs)
            self._refs = (refs, rho)
        return self._refs

    # ------------------------------------------------------------------
    def run_modes(self, modes, steps, warmup):
        """Every requested form on the workload; returns {mode: record}."""
        torch, cfg = self.torch, self.cfg
        results = {}
        fp64_modes = [m for m in modes if m in ("plain", "fp64")]
        mixed = [m for m in modes if m in MIXED]
        m128 = None
        if fp64_modes and not self.streamed:
            m128 = self.resident_m("c128")
        for mode in fp64_modes:
            form, batched = ("gemm", False) if mode == "plain" else ("herk", True)
            try:
                ex, init_ms = self.make("fp64", form, batched)
            except self.lib.ExchangeError as e:
                log(f"[bench] {self.name} {mode}: not run ({e})")
                results[mode] = dict(unsupported=str(e))
                continue
            log(f"[bench] {self.name} {mode}: init {init_ms:.1f} ms")
            if self.streamed:
                ms, energy, per_k = self.timed_streamed(ex, "c128")
                kt = None
            else:
                ms, energy, kt = self.timed(ex, steps, warmup, m128, kernel_timing=(mode != "plain"),
                                            budget_s=SLOW_FORM_BUDGET_S)
            V = self.v_host()
            results[mode] = self.record(ex, ms, init_ms, energy, kt, V, "c128")
            results[mode]["streamed"] = self.streamed
            results[mode]["steps"] = None if self.streamed else self.last_steps
            ex.close()
            log(f"[bench] {self.name} {mode}: {ms:.3f} ms/step, E_x = {energy:.8f}, error {results[mode]['err_eig_ha']}")
        del m128
        torch.cuda.empty_cache()
        if mixed:
            mres = self.resident_m(self.mdt_mixed)
            torch.cuda.synchronize()
            for mode in mixed:
                ex, init_ms = self.make(mode, "herk", True)
                log(f"[bench] {self.name} {mode}: init {init_ms:.1f} ms, autotune + {steps} steps")
                t0 = time.perf_counter()
                ex.matrix_all(mres, self.outs)       # first call: autotuner, graph capture
                torch.cuda.synchronize()
                tune_s = time.perf_counter() - t0
                ms, energy, kt = self.timed(ex, steps, warmup, mres, kernel_timing=True)
                V = self.v_host()
                r = self.record(ex, ms, init_ms, energy, kt, V, "c64" if self.mdt_mixed == "c64" else "c128")
                r["tune_s"] = round(tune_s, 2)
                r["steps"] = self.last_steps
                results[mode] = r
                ex.close()
                log(f"[bench] {self.name} {mode}: {ms:.4f} ms/step, main kernel {kt[0]:.4f} ms, config {r['cfg']}"
                    f"{' (autotuned)' if r['tuned'] else ''}, error {r['err_eig_ha']}")
            del mres
            torch.cuda.empty_cache()
        return results

    def record(self, ex, ms, init_ms, energy, kt, V, ref_kind):
        en, ee = self.errors(V, ref_kind)
        return dict(ms=ms, init_ms=init_ms, energy=energy, kt=kt, err_norm=en, err_eig_ha=ee,
                    flops_nom=ex.query(1), flops_exec=ex.query(2), bytes_alg=ex.query(4),
                    items=int(ex.query(0)), cfg=int(ex.query(3)), tuned=int(ex.query(8)),
                    ws_bytes=ex.query(9), fused=bool(ex.query(10)), V0=V[0])

    # ------------------------------------------------------------------
    def summary(self, results):
        """The workload's headline mode and its figures."""
        cfg = self.cfg
        ok = [m for m in MIXED if m in results and results[m].get("err_eig_ha") is not None
              and results[m]["err_eig_ha"] <= 1e-6]
        head = min(ok, key=lambda m: results[m]["ms"]) if ok else None
        out = {"workload": f"{self.name}: {WORKLOADS[self.name]}"}
        if head is None:
            return None, out
        H = results[head]
        P, F = results.get("plain"), results.get("fp64")
        out.update({
            "mode": head, "value_gflops": round(H["flops_nom"] / (H["ms"] * 1e-3) / 1e9, 3),
            "ms_per_step": round(H["ms"], 5), "kpoints_per_s": round(cfg.n_k / (H["ms"] * 1e-3), 2),
            "pairs_per_s": round(cfg.n_k * cfg.n_q / (H["ms"] * 1e-3), 1),
            "gflops_executed": round(H["flops_exec"] / (H["ms"] * 1e-3) / 1e9, 3),
            "err_eig_ha": H["err_eig_ha"], "err_normwise": H["err_norm"],
            "err_reference": ("oracle V(k=0), all q (tests/golden)" if self.streamed else "oracle, every k"),
            "init_ms": round(H["init_ms"], 2), "kernel_config": H["cfg"], "autotuned": H["tuned"],
        })
        ok_p = P is not None and "ms" in P
        ok_f = F is not None and "ms" in F
        out["speedup_vs_plain_fp64"] = round(P["ms"] / H["ms"], 3) if ok_p else None
        out["batching_factor"] = round(P["ms"] / F["ms"], 3) if ok_p and ok_f else None
        out["precision_factor"] = round(F["ms"] / H["ms"], 3) if ok_f else None
        out["modes"] = {}
        for m, r in results.items():
            if "ms" not in r:
                out["modes"][m] = {"unsupported": r.get("unsupported")}
                continue
            out["modes"][m] = {"ms_per_step": round(r["ms"], 5),
                               "gflops": round(r["flops_nom"] / (r["ms"] * 1e-3) / 1e9, 3),
                               "err_eig_ha": r["err_eig_ha"], "err_normwise": r["err_norm"],
                               "main_kernel_ms": (round(r["kt"][0], 5) if r["kt"] else None),
                               "init_ms": round(r["init_ms"], 1), "config": r["cfg"], "fused": r["fused"],
                               "tuned": r["tuned"], "m_streamed_per_k": r.get("streamed", False),
                               "steps": r.get("steps")}
            if "tune_s" in r:
                out["modes"][m]["tune_s"] = r["tune_s"]
        return head, out

    def roofline(self, results, head):
        """Roofline of the headline mode's dominant kernel, timed live with graph event nodes."""
        H = results[head]
        cfg = self.cfg
        if not (H["kt"] and H["kt"][0] > 0):
            return None
        t_main, t_sparse = H["kt"][0], H["kt"][1]
        esz = 8 if self.mdt_mixed == "c64" else 16
        m_elems = sum(cfg.m_elems(k) for k in range(cfg.n_k))
        e_bytes = sum(16.0 * cfg.n_d(q) ** 2 for q in range(cfg.n_q))
        v_bytes = sum(16.0 * nb * nb for nb in cfg.n_bands)
        if H["fused"]:
            kname = "wide_kernel" if 180 <= H["cfg"] < 200 else "fused_kernel"
            name, t_k = f"{kname} (block-sparse rows, dense rows on MFMA, band contraction; M read once)", t_main
            flops, byts = H["flops_exec"], m_elems * esz + e_bytes + v_bytes
        elif t_main >= t_sparse:
            name, t_k = "tile_kernel (dense rows Y = L^H A on MFMA + band contraction)", t_main
            flops, byts = H["flops_exec"], H["ws_bytes"] + e_bytes + v_bytes
        else:
            name, t_k = "sparse_kernel (block-sparse rows, packs the tile kernel's operands)", t_sparse
            flops, byts = 0.0, m_elems * esz + H["ws_bytes"]
        peak_f = PEAK_TFLOPS[head]
        ridge = peak_f * 1e12 / (HBM_PEAK_GBS * 1e9)
        intensity = flops / byts if byts > 0 else float("inf")
        nprod = {"fp32": 1, "bf16x3": 3, "bf16x6": 6}[head]
        # the binding roof: HBM time of the algorithmic bytes against matrix-core time of the
        # products the mode executes (a split product costs nprod instructions)
        if byts / (HBM_PEAK_GBS * 1e9) >= nprod * flops / (peak_f * 1e12):
            ach = byts / (t_k * 1e-3) / 1e9
            roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(ach / HBM_PEAK_GBS, 5)}
        else:
            ach = flops / (t_k * 1e-3) / 1e12
            roof = {"bound": "mfma", "achieved": round(ach, 3), "peak": peak_f, "unit": "TFLOP/s",
                    "frac": round(ach / peak_f, 5)}
        roof.update({"traffic": _traffic(self.name, head, H["cfg"]), "kernel": name, "kernel_ms": round(t_k, 5),
                     "launches_timed": H["kt"][2], "algorithmic_bytes_per_launch": byts,
                     "algorithmic_flops_per_launch": flops,
                     "intensity_flop_per_byte": round(intensity, 2), "ridge_flop_per_byte": round(ridge, 1),
                     "mfma_frac_algorithmic": round(flops / (t_k * 1e-3) / 1e12 / peak_f, 5),
                     "mfma_frac_executed_products": round(nprod * flops / (t_k * 1e-3) / 1e12 / peak_f, 5)})
        if self.copy_gbs:
            roof["hbm_copy_measured_gbs"] = round(self.copy_gbs, 1)
        return roof

    def measure_copy(self, mib=2048, reps=10):
        """HBM bandwidth of a plain device copy (read + write bytes over event time), beside the
        published 8 TB/s."""
        torch = self.torch
        n = mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=self.dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            dst.copy_(src)
        e1.record()
        e1.synchronize()
        self.copy_gbs = 2.0 * n * 4 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
        del src, dst
        torch.cuda.empty_cache()
        log(f"[bench] device copy: {self.copy_gbs:.0f} GB/s (read + write)")

    # ------------------------------------------------------------------
    def cpu_baseline(self, head_flops_total):
        """The oracle as it stands (dense v, NumPy complex128) on the host cores: a bounded
        sample of the workload's pairs, extrapolated to the whole step by nominal flops."""
        import numpy as np
        from oracle import vx
        cfg, synth = self.cfg, self.synth
        try:
            from threadpoolctl import threadpool_info, threadpool_limits
            threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
        except Exception:
            threadpool_limits = None
            threads = os.cpu_count()
        w = cfg.weights_q()
        budget = 12.0 if self.streamed else 10.0
        # threaded BLAS: pairs of k = 0 in mesh order until the budget is spent
        t_cpu, fl, pairs = 0.0, 0.0, 0
        while (t_cpu < budget or pairs < 1) and pairs < cfg.n_k * cfg.n_q:
            k, qq = divmod(pairs, cfg.n_q)
            v = vx.assemble_v(self.E[qq], self.D, self.C)
            m = synth.m_block(cfg, k, qq)
            t0 = time.perf_counter()
            vx.vx_k([m], [v], [w[qq]])
            t_cpu += time.perf_counter() - t0
            fl += nominal_flops_pair(cfg, k, qq)
            pairs += 1
        gfl = fl / t_cpu / 1e9
        # one thread: the first pair (or part of a full step on the small workloads)
        single = None
        if threadpool_limits is not None:
            v = vx.assemble_v(self.E[0], self.D, self.C)
            m = synth.m_block(cfg, 0, 0)
            with threadpool_limits(limits=1):
                t0 = time.perf_counter()
                vx.vx_k([m], [v], [w[0]])
                t1 = time.perf_counter() - t0
            single = {"value": round(nominal_flops_pair(cfg, 0, 0) / t1 / 1e9, 3), "cores": 1,
                      "sample": "pair (k=0, q=0) with the BLAS limited to one thread"}
        full_s = head_flops_total / (gfl * 1e9)
        return {"value": round(gfl, 3), "unit": "GFLOP/s", "cores": threads, "kind": "oracle",
                "sample": f"{pairs} (k, q) pairs of the {cfg.n_k * cfg.n_q} (k = 0 first, q in mesh order) with the "
                          f"dense-v NumPy oracle ({t_cpu:.1f} s); GFLOP counted as the method's nominal flops",
                "step_s_extrapolated": round(full_s, 1),
                "extrapolation": "whole step (all k, all q) by nominal flops from the sample",
                "single_thread": single}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c4", choices=sorted(WORKLOADS))
    ap.add_argument("--also", default="c3,c2", help="workloads reported beside the headline (comma list)")
    ap.add_argument("--modes", default="plain,fp64,fp32,bf16x3,bf16x6")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-legs", action="store_true", help="skip the widening-row legs on the Si-like workload")
    ap.add_argument("--only", default=None, help="one mode of the headline workload only (profiling runs)")
    ap.add_argument("--learned", action="store_true",
                    help="also run the learned extrapolator's 30 outer iterations on the whole ZnO-like workload")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device-to-device 3 times (scales HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the exchange path here is built and timed on a "
              "single MI355X (sharding the q sum over GPUs, with one all-reduce of the FP64 partial V, is not run).",
              file=sys.stderr)
        return 2

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

    B = Bench(args, torch, lib, synth)
    modes = [args.only] if args.only else [m for m in args.modes.split(",") if m]
    B.setup(args.workload)
    results = B.run_modes(modes, args.steps, args.warmup)
    head, summ = B.summary(results)
    if head is None:
        head = next((m for m in ("fp64", "plain") if m in results and "ms" in results[m]), None)
    if head is None:       # no mode met the error target and no FP64 form ran: the fastest one, flagged
        head = min((m for m in results if "ms" in results[m]), key=lambda m: results[m]["ms"])
        log(f"[bench] no mode of {args.workload} met the 1e-6 Ha target; reporting {head}")
    H = results[head]
    roof = B.roofline(results, head) if head in MIXED else None
    cpu = None
    if not args.no_cpu and not args.only:
        cpu = B.cpu_baseline(H["flops_nom"])
        log(f"[bench] cpu oracle: {cpu['value']} GFLOP/s on {cpu['cores']} threads "
            f"(single thread {cpu['single_thread'] and cpu['single_thread']['value']}), "
            f"step extrapolated {cpu['step_s_extrapolated']} s")
    value = H["flops_nom"] / (H["ms"] * 1e-3) / 1e9
    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "GFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(H["ms"], 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPE[head], "data": "synthetic (seeded SplitMix64/Box-Muller M drawn on the GPU, synthetic PD "
                                      "Coulomb blocks)",
        "config": {"workload": summ["workload"], "mode": head,
                   "form": "cholesky-herk, one persistent launch over all (k, q) in a HIP graph",
                   "m_dtype": B.mdt_mixed, "kernel_config": H["cfg"], "autotuned": H["tuned"]},
        "kpoints_per_s": round(B.cfg.n_k / (H["ms"] * 1e-3), 2),
        "pairs_per_s": round(B.cfg.n_k * B.cfg.n_q / (H["ms"] * 1e-3), 1),
        "gflops_executed": round(H["flops_exec"] / (H["ms"] * 1e-3) / 1e9, 3),
        "err_eig_ha": H["err_eig_ha"], "err_normwise": H["err_norm"],
        "err_reference": summ.get("err_reference"),
        "init_ms": round(H["init_ms"], 2),
        "roofline": roof, "cpu_baseline": cpu,
        "modes": summ.get("modes"),
        "speedup_vs_plain_fp64": summ.get("speedup_vs_plain_fp64"),
        "batching_factor": summ.get("batching_factor"),
        "precision_factor": summ.get("precision_factor"),
    }
    if args.workload == "c2" and not args.no_legs and not args.only and head in MIXED:
        out.update(c2_legs(B, head, H["ms"], args))
    if not args.only:
        for name in [w for w in args.also.split(",") if w and w != args.workload]:
            B2 = Bench(args, torch, lib, synth)
            B2.setup(name)
            steps = args.steps if name != "c2" else max(args.steps, 50)
            warm = args.warmup if name != "c2" else max(args.warmup, 10)
            res2 = B2.run_modes(modes, steps, warm)
            h2, s2 = B2.summary(res2)
            if h2 is not None:
                s2["roofline"] = B2.roofline(res2, h2)
            if name == "c2" and not args.no_legs and h2 is not None:
                s2.update(c2_legs(B2, h2, res2[h2]["ms"], args))
            out[name] = s2
    if args.learned and not args.only:
        out["learned_c3"] = learned_leg(torch, lib, synth)
    print(json.dumps(out))
    return 0


def learned_leg(torch, lib, synth):
    """The learned extrapolator on the whole ZnO-like workload (21 k x 144 q): 30 synthetic outer
    iterations, 10 training pairs, the exact FP64 HERK path every 5th iteration as the judge."""
    import numpy as np
    import synth.scf as scf
    from paper_1003_0524_amd import learned
    cfg = synth.make_config("c3")
    torch.cuda.empty_cache()
    E, D, C = synth.coulomb_blocks(cfg)
    ex = lib.Exchange(cfg.n_bands, cfg.n_pw, cfg.ch_nrad, cfg.n_occ, E, D, C, w_q=cfg.weights_q(),
                      precision="fp64", form="herk", batched=True)
    stamps = []
    try:
        feed = scf.make_feed_device(cfg, 30, torch.device("cuda"))

        def on_iter(r):
            torch.cuda.synchronize()
            stamps.append((r.t, r.exact, time.perf_counter()))
            log(f"[bench] learned t={r.t} {r.used}" + (f" err {r.err_pred:.3e} stale {r.err_stale:.3e}" if r.judged else ""))
        xp = learned.Extrapolator(ex, n_blk=cfg.n_bands[0], epochs=1500, epochs_ft=300)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        recs, xp, _ = learned.run_outer(ex, feed, n_iter=30, tau=1e-4, xp=xp, on_iter=on_iter)
    finally:
        ex.close()
        feed = None
        torch.cuda.empty_cache()
    dts = [(e, b - a) for (_, _, a), (_, e, b) in zip([(0, True, t0)] + stamps[:-1], stamps)]
    judged = [r for r in recs if r.judged]
    return {"workload": "c3 (all 21 k x 144 q)", "n_blk": cfg.n_bands[0], "iterations": len(recs), "exact": sum(r.exact for r in recs),
            "predicted": sum(not r.exact for r in recs), "tau_ha": 1e-4,
            "seconds_total": round(stamps[-1][2] - t0, 3),
            "seconds_per_predicted_iteration": round(float(np.mean([d for e, d in dts if not e])), 4)
            if any(not e for e, _ in dts) else None,
            "judged": [{"t": r.t, "err_pred": r.err_pred, "err_stale": r.err_stale, "err_ridge": r.err_ridge,
                        "err_pred_block": r.err_pred_block, "err_stale_block": r.err_stale_block,
                        "accepted": r.accepted} for r in judged]}


def c2_legs(B, head, head_ms, args):
    """Widening rows on the Si-like workload: inversion-symmetric variant, EIBZ-restricted q sum,
    Gamma-point term and back-transform."""
    import numpy as np
    from oracle import precision as pr
    from oracle import vx
    torch, cfg, synth, dev = B.torch, B.cfg, B.synth, B.dev
    mdt = np.complex128
    legs = {}
    steps, warm = max(args.steps, 50), max(args.warmup, 10)
    mesh = tuple(len(np.unique(np.round(cfg.q_frac[:, i], 12))) for i in range(3))
    ex, _ = B.make(head, "herk", True)
    c_gamma = ex.gamma_term(cfg.recip(), mesh, 0.005, apply=False)
    kms = []
    for _ in range(5):
        ex.gamma_term(cfg.recip(), mesh, 0.005, apply=False)
        kms.append(ex.gamma_kernel_ms()[0])
    n_terms = ex.gamma_kernel_ms()[1]
    legs["gamma_term"] = {"C": c_gamma, "beta": 0.005, "mesh": list(mesh), "terms": n_terms,
                          "kernel_ms": round(float(np.mean(kms)), 5),
                          "terms_per_s": round(n_terms / (float(np.mean(kms)) * 1e-3), 1)}
    ex.close()
    # back-transform of V(k=0) (FP64 HERK context) to n_G LAPW functions (synthetic Z = S c)
    M128 = B.resident_m("c128")
    ex, _ = B.make("fp64", "herk", True)
    ex.matrix_all(M128, B.outs)
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
    legs["back_transform"] = btx
    ex.close()
    # inversion-symmetric variant in the headline's precision
    Mr = [torch.from_numpy(synth.m_all_real_packed(cfg, k, mdt)).to(dev) for k in range(cfg.n_k)]
    exr, _ = B.make(head, "herk", True, inversion=True)
    ms_r, _, kt_r = B.timed(exr, steps, warm, Mr, kernel_timing=True)
    Vr = B.v_host()
    nom_r, cfg_r = exr.query(1), int(exr.query(3))
    exr.close()
    Er, Dr, Cr = synth.coulomb_blocks_real(cfg)
    vr = [vx.assemble_v(Er[q], Dr, Cr) for q in range(cfg.n_q)]
    refs_r = [vx.vx_k([synth.m_block_real(cfg, k, q) for q in range(cfg.n_q)], vr, cfg.weights_q())
              for k in range(cfg.n_k)]
    rho_r = max(np.abs(np.linalg.eigvalsh(r.real)).max() for r in refs_r)
    legs["inversion_variant"] = {
        "mode": head, "ms_per_step": round(ms_r, 5), "main_kernel_ms": round(kt_r[0], 5),
        "gflops_nominal_real": round(nom_r / (ms_r * 1e-3) / 1e9, 3),
        "kpoints_per_s": round(cfg.n_k / (ms_r * 1e-3), 1),
        "speedup_vs_complex": round(head_ms / ms_r, 3), "config": cfg_r,
        "err_normwise": max(pr.normwise_error(a, b) for a, b in zip(Vr, refs_r)),
        "err_eig_ha": max(pr.normalised_eig_error(a, b, rho_r) for a, b in zip(Vr, refs_r))}
    # q sum over the extended irreducible wedge EIBZ(k) of each irreducible k
    from paper_1003_0524_amd import symmetry as sy
    ops = sy.point_group(cfg.lattice)
    k_idx, _ = sy.irreducible(cfg.q_frac, ops)
    if len(k_idx) == cfg.n_k:
        w_kq = np.stack([sy.eibz_weights(cfg.q_frac[i], cfg.q_frac, ops, cfg.weights_q())[0] for i in k_idx])
        Me = [synth.m_all_device(cfg, k, "c128", dev, keep=w_kq[k] != 0) for k in range(cfg.n_k)]
        exe, _ = B.make(head, "herk", True, w_kq=w_kq)
        ms_e, _, kt_e = B.timed(exe, steps, warm, Me, kernel_timing=True)
        Ve = B.v_host()
        cfg_e, fused_e, split_e = int(exe.query(3)), bool(exe.query(10)), int(exe.query(14))
        exe.close()
        E, D, C = B.E, B.D, B.C
        v = [vx.assemble_v(E[q], D, C) for q in range(cfg.n_q)]
        refs_e = []
        for k in range(cfg.n_k):
            keep = [q for q in range(cfg.n_q) if w_kq[k, q] != 0]
            refs_e.append(vx.vx_k([synth.m_block(cfg, k, q) for q in keep], [v[q] for q in keep], w_kq[k, keep]))
        n_pairs = int(np.count_nonzero(w_kq))
        legs["eibz_q_sum"] = {
            "mode": head, "pairs": n_pairs, "pairs_full_mesh": cfg.n_k * cfg.n_q,
            "ms_per_step": round(ms_e, 5), "main_kernel_ms": round(kt_e[0], 5),
            "sparse_kernel_ms": round(kt_e[1], 5), "config": cfg_e, "fused": fused_e,
            "item_split": {0: "pair", 1: "pair x n'' chunk", 2: "pair x n'' chunk x row part"}.get(split_e, split_e),
            "kpoints_per_s": round(cfg.n_k / (ms_e * 1e-3), 1),
            "speedup_vs_full_mesh": round(head_ms / ms_e, 3),
            "note": "V(k) summed over EIBZ(k) only; the rotation over the little group LG(k) that completes "
                    "the full sum (done in the LAPW basis) is not included in the time",
            "err_normwise": max(pr.normwise_error(a, b) for a, b in zip(Ve, refs_e))}
    return legs


if __name__ == "__main__":
    sys.exit(main())
