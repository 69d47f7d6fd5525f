"""The device twin of the M generator draws the host generator's values (GPU).

Sampled (k, q) blocks of several workloads -- the SrTiO3-like and ZnO-like ones at
their full per-pair sizes included -- against ``synth.m_block``: complex128 to a few
units in the last place of float64 (the device log, sin, cos and exp are not the
host's), complex64 equal to the host values rounded to complex64 except where such
a last-place difference crosses a rounding boundary (one binary32 unit at most).
"""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CASES = [("tiny", 1, 2), ("ragged", 2, 5), ("c2", 3, 17), ("c3", 0, 0), ("c3", 20, 143), ("c4", 0, 0),
         ("c4", 19, 215), ("c4", 7, 101)]


@pytest.mark.parametrize("name,k,q", CASES)
def test_device_block_matches_host(name, k, q):
    cfg = synth.make_config(name)
    print(f"[synth-device] {name} k={k} q={q} N_MB={cfg.n_mb(q)}", flush=True)
    host = synth.m_block(cfg, k, q).ravel()
    dev = synth.m_block_device(cfg, k, q, "c128").cpu().numpy()
    assert dev.shape == host.shape
    scale = np.max(np.abs(host))
    assert np.max(np.abs(dev - host)) <= 1e-15 * scale
    dev64 = synth.m_block_device(cfg, k, q, "c64").cpu().numpy()
    host64 = host.astype(np.complex64)
    diff = dev64 != host64
    assert np.count_nonzero(diff) <= max(2, host.size // 10**6)
    for part in (np.real, np.imag):
        a, b = part(dev64), part(host64)
        assert np.all(np.abs(a.astype(np.float64) - b) <= np.spacing(np.abs(b).astype(np.float32)) * 1.0)


def test_all_blocks_of_k_in_mesh_order():
    cfg = synth.make_config("ragged")
    for k in range(cfg.n_k):
        dev = synth.m_all_device(cfg, k, "c128").cpu().numpy()
        host = synth.m_all(cfg, k)
        assert np.max(np.abs(dev - host)) <= 1e-15 * np.max(np.abs(host))
    # only the kept blocks, in mesh order
    keep = np.array([q % 2 == 0 for q in range(cfg.n_q)])
    dev = synth.m_all_device(cfg, 1, "c128", keep=keep).cpu().numpy()
    host = np.concatenate([synth.m_block(cfg, 1, q).ravel() for q in range(cfg.n_q) if keep[q]])
    assert np.max(np.abs(dev - host)) <= 1e-15 * np.max(np.abs(host))
