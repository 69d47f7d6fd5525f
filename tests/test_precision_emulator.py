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
    got = pr.vx_k_emulated(mb, L, cfg.weights_q(), "fp64")
    assert pr.normwise_error(got, ref) < 1e-13
    e32 = pr.normwise_error(pr.vx_k_emulated(mb, L, cfg.weights_q(), "fp32"), ref)
    e16 = pr.normwise_error(pr.vx_k_emulated(mb, L, cfg.weights_q(), "bf16x3"), ref)
    assert 1e-10 < e32 < 1e-6 and e32 < e16 < 1e-4


def test_three_way_split_error_bound():
    rng = np.random.default_rng(2)
    x = rng.standard_normal(100000)
    hi, mid, lo = pr.split3_bf16(x)
    assert np.all(np.abs(x - hi - mid - lo) <= 2.0 ** -24 * np.abs(x))


def test_sequential_binary32_product_is_exact_on_small_integers():
    """Chunked binary32 complex products: exact when every partial sum is an integer
    below 2^24 (and every piece of a bf16 split is exact), for any chunk size."""
    rng = np.random.default_rng(5)
    a = rng.integers(-8, 9, (7, 45)) + 1j * rng.integers(-8, 9, (7, 45))
    b = rng.integers(-8, 9, (45, 5)) + 1j * rng.integers(-8, 9, (45, 5))
    exact = a @ b
    for n in (1, 2, 3):
        for chunk in (1, 4, 32, 64):
            assert np.array_equal(pr._cmm32_seq(a, b, n, chunk), exact)


def test_sequential_binary32_accumulation_error_grows_with_k():
    """Summing many terms one chunk at a time in binary32 loses more than the same
    sum taken in one float64 pass; the emulated error must show it."""
    rng = np.random.default_rng(6)
    K = 4096
    a = (rng.standard_normal((1, K)) + 1.0).astype(np.complex128)
    b = np.ones((K, 1), dtype=np.complex128)
    ref = (a @ b)[0, 0]
    got = pr._cmm32_seq(a, b, 1, 4)[0, 0]
    assert abs(got - ref) > 0.0
    # bounded by the sequential-summation bound (K/4 additions of relative error 2^-24)
    assert abs(got - ref) <= (K / 4) * 2.0 ** -24 * np.sum(np.abs(a))
