"""Pins of the reduced-precision emulator used to set mixed-precision tolerances."""
import numpy as np
import pytest
import torch

import synth
from oracle import chol, precision as pr, vx


def test_bf16_rne_matches_torch_conversion():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-6, 6, 20000),
                        # exact ties: 1 + (2j+1) 2^-8 round to even
                        1.0 + (2 * np.arange(50) + 1) * 2.0 ** -8]).astype(np.float32)
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    got = pr.bf16_rne(x.astype(np.float64))
    assert np.array_equal(got, want)


def test_split_error_bound():
    rng = np.random.default_rng(1)
    x = rng.standard_normal(100000)
    hi, lo = pr.split_bf16(x)
    assert np.all(np.abs(x - hi) <= 2.0 ** -8 * np.abs(x))
    assert np.all(np.abs(x - hi - lo) <= 2.0 ** -16 * np.abs(x))


def test_emulator_fp64_mode_is_oracle():
    cfg = synth.make_config("small")
    E, D, C = synth.coulomb_blocks(cfg)
    v = [vx.assemble_v(E[q], D, C) for q in range(cfg.n_q)]
    L = [chol.cholesky(a) for a in v]
    mb = [synth.m_block(cfg, 0, q) for q in range(cfg.n_q)]
    ref = vx.vx_k(mb, v, cfg.weights_q())
    got = pr.vx_k_emulated(mb, L, cfg.weights_q(), "fp64", cfg.n_s)
    assert pr.normwise_error(got, ref) < 1e-13
    e32 = pr.normwise_error(pr.vx_k_emulated(mb, L, cfg.weights_q(), "fp32", cfg.n_s), ref)
    e6 = pr.normwise_error(pr.vx_k_emulated(mb, L, cfg.weights_q(), "bf16x6", cfg.n_s), ref)
    e16 = pr.normwise_error(pr.vx_k_emulated(mb, L, cfg.weights_q(), "bf16x3", cfg.n_s), ref)
    # 24-bit operands (fp32, bf16x6) against 16-bit ones (bf16x3)
    assert 1e-10 < e32 < 1e-6 and 1e-10 < e6 < 1e-6 and max(e32, e6) < e16 < 1e-4


def test_three_way_split_error_bound():
    rng = np.random.default_rng(2)
    x = rng.standard_normal(100000)
    hi, mid, lo = pr.split3_bf16(x)
    assert np.all(np.abs(x - hi - mid - lo) <= 2.0 ** -24 * np.abs(x))
