"""Pins of the back-transform oracle (Sec. III.A, eq. "APW trafo").

  * element-by-element loops on tiny sizes;
  * the back-transform inverts the band projection: with overlap S (Hermitian
    positive definite) and eigenvectors c, c^H S c = 1, projecting V_GG back
    with c gives V again (c^H V_GG c = V);
  * Hermitian V gives Hermitian V_GG of rank <= n_b.
"""
import numpy as np
import pytest

from oracle import backx


def _hpd(rng, n):
    x = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    return x @ x.conj().T / n + np.eye(n)


def _herm(rng, n):
    x = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    return (x + x.conj().T) / 2


def test_matches_loops():
    rng = np.random.default_rng(1)
    Z = rng.standard_normal((5, 3)) + 1j * rng.standard_normal((5, 3))
    V = rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3))
    assert np.allclose(backx.back_transform(Z, V), backx.back_transform_loops(Z, V), rtol=0, atol=1e-13)


def test_inverts_the_band_projection():
    rng = np.random.default_rng(2)
    nG, nb = 40, 7
    S = _hpd(rng, nG)
    w, U = np.linalg.eigh(S)
    S_inv_half = U @ np.diag(w ** -0.5) @ U.conj().T
    Q, _ = np.linalg.qr(rng.standard_normal((nG, nb)) + 1j * rng.standard_normal((nG, nb)))
    c = S_inv_half @ Q                                   # c^H S c = Q^H Q = 1
    assert np.allclose(c.conj().T @ S @ c, np.eye(nb), atol=1e-12)
    V = _herm(rng, nb)
    VGG = backx.back_transform(S @ c, V)
    assert np.allclose(c.conj().T @ VGG @ c, V, rtol=0, atol=1e-11 * np.abs(V).max())


def test_hermitian_and_rank():
    rng = np.random.default_rng(3)
    Z = rng.standard_normal((30, 6)) + 1j * rng.standard_normal((30, 6))
    VGG = backx.back_transform(Z, _herm(rng, 6))
    assert np.allclose(VGG, VGG.conj().T, atol=1e-12 * np.abs(VGG).max())
    assert np.linalg.matrix_rank(VGG, tol=1e-10 * np.abs(VGG).max()) <= 6
