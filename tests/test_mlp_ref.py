"""Pins of the float64 MLP reference and of the extrapolator encoding (CPU).

Each check compares the oracle with something other than itself: central
finite differences of the loss, Adam's closed-form first step, limits of the
network (zero weights, small inputs, odd symmetry), algebraic identities of the
encoding, Weyl's bound for the judge, and exact recovery by the ridge fit.
"""
import numpy as np
import pytest

import synth
from oracle import learned, mlp

I, H, O = 12, 16, 9


def _theta(seed=3):
    return mlp.init_params(I, H, O, seed, synth.splitmix64_stream)


def _data(n=7, seed=5):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, I)), rng.standard_normal((n, O))


def test_init_matches_scalar_splitmix64_and_bounds():
    theta = _theta(11)
    W1, b1, W2, b2, W3, b3 = mlp.unpack(theta, I, H, O)
    # entry 5 of W1 (flat index 5) and entry 2 of W3 from the scalar generator
    offs, _, _ = mlp.layout(I, H, O)
    for flat, fan in ((5, I), (offs[4] + 2, H)):
        u = (synth.sm_int(11, flat) >> 11) / 2.0 ** 53
        assert theta[flat] == pytest.approx((2 * u - 1) / np.sqrt(fan), abs=1e-15)
    assert np.all(b1 == 0) and np.all(b2 == 0) and np.all(b3 == 0)
    assert np.max(np.abs(W1)) <= 1 / np.sqrt(I) and np.max(np.abs(W2)) <= 1 / np.sqrt(H)


def test_gradient_matches_central_differences():
    theta = _theta() * 1.7
    theta[mlp.layout(I, H, O)[0][1]:][:H] += 0.1       # non-zero b1
    X, T = _data()
    L, g = mlp.grad(theta, X, T, I, H, O)
    assert L == pytest.approx(mlp.loss(theta, X, T, I, H, O), rel=1e-15)
    rng = np.random.default_rng(0)
    idx = np.concatenate([rng.choice(theta.size, 40, replace=False),
                          [0, theta.size - 1, mlp.layout(I, H, O)[0][3]]])
    h = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (mlp.loss(tp, X, T, I, H, O) - mlp.loss(tm, X, T, I, H, O)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1e-3, abs(g[i])) + 1e-10, (i, fd, g[i])


def test_directional_derivative_matches_finite_difference():
    theta = _theta()
    X, T = _data(n=5, seed=9)
    _, g = mlp.grad(theta, X, T, I, H, O)
    d = np.random.default_rng(2).standard_normal(theta.size)
    h = 1e-6
    fd = (mlp.loss(theta + h * d, X, T, I, H, O) - mlp.loss(theta - h * d, X, T, I, H, O)) / (2 * h)
    assert fd == pytest.approx(g @ d, rel=1e-7)


def test_adam_first_step_closed_form():
    # zero moments, t = 1: m_hat = g and v_hat = g^2, so the step is lr * g / (|g| + eps)
    theta = _theta()
    g = np.random.default_rng(4).standard_normal(theta.size) * 1e-3
    opt = mlp.Adam(theta.size, lr=0.01)
    new = opt.step(theta, g)
    assert np.allclose(theta - new, 0.01 * g / (np.abs(g) + mlp.EPS), rtol=1e-12, atol=0)
    # second step with the same gradient: moments still give m_hat = g, v_hat = g^2
    new2 = opt.step(new, g)
    assert np.allclose(new - new2, 0.01 * g / (np.abs(g) + mlp.EPS), rtol=1e-9, atol=0)


def test_zero_weights_give_output_bias():
    theta = np.zeros(mlp.layout(I, H, O)[2])
    b3 = np.arange(O, dtype=float)
    theta[-O:] = b3
    X, _ = _data()
    y, _ = mlp.forward(theta, X, I, H, O)
    assert np.array_equal(y, np.tile(b3, (X.shape[0], 1)))


def test_odd_symmetry_without_biases():
    theta = _theta()
    X, _ = _data()
    y1, _ = mlp.forward(theta, X, I, H, O)
    y2, _ = mlp.forward(theta, -X, I, H, O)
    assert np.allclose(y1, -y2, rtol=0, atol=1e-15)


def test_small_input_limit_is_product_of_weights():
    theta = _theta()
    W1, _, W2, _, W3, _ = mlp.unpack(theta, I, H, O)
    x = np.random.default_rng(8).standard_normal((1, I))
    eps = 1e-6
    y, _ = mlp.forward(theta, eps * x, I, H, O)
    lin = (W3 @ (W2 @ (W1 @ x[0])))
    assert np.allclose(y[0] / eps, lin, rtol=1e-9, atol=1e-10)


def test_training_reduces_loss():
    theta = _theta()
    X, T = _data(n=20)
    L0 = mlp.loss(theta, X, T, I, H, O)
    _, L = mlp.train(theta, X, T, I, H, O, epochs=200, lr=3e-3)
    assert L < 0.2 * L0


# ---------------------------------------------------------------- encoding ---
def _herm(n, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    return A + A.conj().T


def test_encode_decode_roundtrip_and_layout():
    Hm = _herm(5, 1)
    y = learned.encode(Hm)
    assert y.size == 25
    assert np.allclose(learned.decode(y, 5), Hm, atol=0, rtol=0)
    R = y.reshape(5, 5)
    assert R[1, 3] == Hm[1, 3].real and R[3, 1] == Hm[1, 3].imag and R[2, 2] == Hm[2, 2].real


def test_expand_of_projection_with_full_basis_is_exact():
    n = 6
    V = -np.eye(n) * np.arange(1, n + 1) + 0.1 * _herm(n, 2)
    dV = 0.01 * _herm(n, 3)
    B = learned.basis(V, n)                     # unitary
    y = learned.project(dV, B, 1.0 / 0.37)
    assert np.allclose(learned.expand(V, B, y, 0.37), V + dV, rtol=0, atol=1e-14)


def test_partial_basis_gives_projected_change():
    n, nb = 7, 3
    V = -np.diag(np.arange(1.0, n + 1)) + 0.05 * _herm(n, 4)
    dV = 0.01 * _herm(n, 5)
    B = learned.basis(V, nb)
    w = np.linalg.eigvalsh(V)
    assert np.allclose(B.conj().T @ V @ B, np.diag(w[:nb]), atol=1e-13)
    P = B @ B.conj().T
    assert np.allclose(learned.expand(V, B, learned.project(dV, B, 1.0), 1.0), V + P @ dV @ P, atol=1e-14)


def test_judge_zero_for_equal_and_weyl_bound():
    n = 8
    V = -np.diag(np.arange(1.0, n + 1))
    dV = 1e-3 * _herm(n, 6)
    assert learned.judge_error(V, V, 4, 2.0) == 0.0
    e = learned.judge_error(V + dV, V, 4, 2.0)
    assert 0 < e <= np.linalg.norm(dV, 2) / 2.0 + 1e-15


def test_dp_vector_layout():
    M = np.array([[1 + 2j, 3 + 4j], [5 + 6j, 7 + 8j]])
    v = learned.dp_vector([M, 2 * M])
    # column-major: M[0,0], M[1,0], M[0,1], M[1,1]
    assert list(v[:8]) == [1, 2, 5, 6, 3, 4, 7, 8]
    assert np.array_equal(v[8:], 2 * v[:8])


def test_sketch_signs_and_norm():
    v = np.zeros(50)
    v[17] = -3.0
    s, nrm = learned.sketch(v, 16, 99, synth.splitmix64_stream)
    assert nrm == 3.0
    for i in (0, 7, 15):
        sign = -1.0 if (synth.sm_int(99, i * 50 + 17) >> 63) else 1.0
        assert s[i] == pytest.approx(-sign / 4.0, abs=1e-15)
    # Johnson-Lindenstrauss-type behaviour: |S v| ~ |v| on average
    rng = np.random.default_rng(0)
    norms = [np.linalg.norm(learned.sketch(rng.standard_normal(400), 64, 7, synth.splitmix64_stream)[0])
             for _ in range(30)]
    assert abs(np.mean(np.square(norms)) - 1.0) < 0.15


def test_ridge_recovers_affine_map():
    rng = np.random.default_rng(1)
    X = rng.standard_normal((40, 6))
    W = rng.standard_normal((6, 3))
    b = rng.standard_normal(3)
    Y = X @ W + b
    Wf = learned.ridge_fit(X, Y, 1e-12)
    assert np.allclose(Wf[:6], W, atol=1e-8) and np.allclose(Wf[6], b, atol=1e-8)
