"""Float64 reference of the learned V^x extrapolator's network -- TEST INFRASTRUCTURE ONLY.

The paper keeps V^x fixed during the inner density iterations and recomputes it
only per outer step (Sec. IV, nested self-consistency). The extension predicts
the change of V^x between exact evaluations with a small multilayer perceptron;
this module is the plain float64 statement of that network and its training
step, against which the GPU kernels are checked.

Network (two hidden layers of width H, tanh activation, linear output):

    h1 = tanh(W1 x + b1),   h2 = tanh(W2 h1 + b2),   y = W3 h2 + b3

with W1: H x I, W2: H x H, W3: O x H (row-major), and the flat parameter vector
ordered [W1, b1, W2, b2, W3, b3].

Loss: mean squared error over the batch and the outputs,
    L = 1/(n O) * sum_{s,o} (y_so - t_so)^2.

Adam (Kingma & Ba 2015, Algorithm 1) with beta1 = 0.9, beta2 = 0.999,
eps = 1e-8 and bias correction; the step counter starts at 1.

Initial weights: W_l entries (2u - 1)/sqrt(fan_in) with u the top 53 bits of
the SplitMix64 output at the entry's index in the flat vector, divided by 2^53;
biases zero.
"""
from __future__ import annotations

import numpy as np

BETA1 = 0.9
BETA2 = 0.999
EPS = 1e-8


def layout(I: int, H: int, O: int):
    """Offsets and shapes of (W1, b1, W2, b2, W3, b3) inside the flat vector."""
    shapes = [(H, I), (H,), (H, H), (H,), (O, H), (O,)]
    offs, o = [], 0
    for s in shapes:
        offs.append(o)
        o += int(np.prod(s))
    return offs, shapes, o


def unpack(theta: np.ndarray, I: int, H: int, O: int):
    offs, shapes, n = layout(I, H, O)
    assert theta.size == n
    return [theta[o:o + int(np.prod(s))].reshape(s) for o, s in zip(offs, shapes)]


def pack(parts) -> np.ndarray:
    return np.concatenate([np.asarray(p, dtype=np.float64).ravel() for p in parts])


def init_params(I: int, H: int, O: int, seed: int, stream) -> np.ndarray:
    """Initial parameters; ``stream(seed, start, count)`` is the SplitMix64 counter stream."""
    offs, shapes, n = layout(I, H, O)
    theta = np.zeros(n)
    for li, fan_in in ((0, I), (2, H), (4, H)):
        o, cnt = offs[li], int(np.prod(shapes[li]))
        x = stream(seed, o, cnt)
        u = (x >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
        theta[o:o + cnt] = (2.0 * u - 1.0) / np.sqrt(fan_in)
    return theta


def forward(theta: np.ndarray, X: np.ndarray, I: int, H: int, O: int):
    """Outputs Y (n x O) and the activations needed by the backward pass."""
    W1, b1, W2, b2, W3, b3 = unpack(theta, I, H, O)
    h1 = np.tanh(X @ W1.T + b1)
    h2 = np.tanh(h1 @ W2.T + b2)
    y = h2 @ W3.T + b3
    return y, (X, h1, h2)


def loss(theta: np.ndarray, X: np.ndarray, T: np.ndarray, I: int, H: int, O: int) -> float:
    y, _ = forward(theta, X, I, H, O)
    return float(np.mean((y - T) ** 2))


def grad(theta: np.ndarray, X: np.ndarray, T: np.ndarray, I: int, H: int, O: int):
    """(loss, dL/dtheta) by the chain rule, layer by layer from the output back."""
    W1, b1, W2, b2, W3, b3 = unpack(theta, I, H, O)
    y, (x, h1, h2) = forward(theta, X, I, H, O)
    n = X.shape[0]
    L = float(np.mean((y - T) ** 2))
    dy = 2.0 * (y - T) / (n * O)              # dL/dy
    gW3 = dy.T @ h2
    gb3 = dy.sum(axis=0)
    dz2 = (dy @ W3) * (1.0 - h2 ** 2)         # through tanh: d tanh(z)/dz = 1 - tanh(z)^2
    gW2 = dz2.T @ h1
    gb2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2) * (1.0 - h1 ** 2)
    gW1 = dz1.T @ x
    gb1 = dz1.sum(axis=0)
    return L, pack([gW1, gb1, gW2, gb2, gW3, gb3])


class Adam:
    """Adam state (first and second moments, step counter) for a flat vector."""

    def __init__(self, n: int, lr: float):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0
        self.lr = lr

    def step(self, theta: np.ndarray, g: np.ndarray) -> np.ndarray:
        self.t += 1
        self.m = BETA1 * self.m + (1.0 - BETA1) * g
        self.v = BETA2 * self.v + (1.0 - BETA2) * g * g
        mhat = self.m / (1.0 - BETA1 ** self.t)
        vhat = self.v / (1.0 - BETA2 ** self.t)
        return theta - self.lr * mhat / (np.sqrt(vhat) + EPS)


def train(theta: np.ndarray, X: np.ndarray, T: np.ndarray, I: int, H: int, O: int,
          epochs: int, lr: float):
    """Full-batch Adam for ``epochs`` steps; returns (theta, loss at the last step)."""
    opt = Adam(theta.size, lr)
    L = np.nan
    for _ in range(epochs):
        L, g = grad(theta, X, T, I, H, O)
        theta = opt.step(theta, g)
    return theta, L
