"""Write the oracle's V^x at the first irreducible k of the ZnO-like (c3) and
SrTiO3-like (c4) workloads, for the full-size checks of the tests and the benchmark.

    python tests/golden/make_vx_golden.py [c3] [c4]

The whole q sum of one k at these sizes (144 / 216 q points, N_MB up to 1399 / 2600,
dense v) costs 1.5 / 18 TFLOP in the float64 oracle: minutes on a host, too long to
repeat inside a test or a benchmark run. Calls only ``oracle`` (the definition, Sec.
III.C eq. "vec-mat-vec", dense Coulomb matrix) and ``synth`` (the seeded inputs).

For each workload two matrices are written, both for k = 0 with every q:
  vx_<name>_k0_c128.npy -- from M drawn in float64 (the input of the FP64 forms);
  vx_<name>_k0_c64.npy  -- from the same M rounded to complex64 and widened (the input
                           the reduced-precision forms are handed).
The q sum is taken one q at a time (V = sum_q of the oracle's single-q result).
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import vx  # noqa: E402


def golden_path(name: str, dtype: str) -> str:
    return os.path.join(HERE, f"vx_{name}_k0_{dtype}.npy")


def compute(name: str, k: int = 0):
    cfg = synth.make_config(name)
    E, D, C = synth.coulomb_blocks(cfg)
    w = cfg.weights_q()
    nb = cfg.n_bands[k]
    V128 = np.zeros((nb, nb), np.complex128)
    V64 = np.zeros((nb, nb), np.complex128)
    t0 = time.time()
    for q in range(cfg.n_q):
        v = vx.assemble_v(E[q], D, C)
        m = synth.m_block(cfg, k, q)
        V128 += vx.vx_k([m], [v], [w[q]])
        V64 += vx.vx_k([m.astype(np.complex64).astype(np.complex128)], [v], [w[q]])
        if q % 24 == 23:
            print(f"[golden] {name}: {q + 1}/{cfg.n_q} q, {time.time() - t0:.0f} s", flush=True)
    return V128, V64


def main(names):
    for name in names:
        V128, V64 = compute(name)
        np.save(golden_path(name, "c128"), V128)
        np.save(golden_path(name, "c64"), V64)
        print(f"[golden] {name}: wrote {golden_path(name, 'c128')} and {golden_path(name, 'c64')}", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["c3", "c4"])
