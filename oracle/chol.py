"""Cholesky re-arrangement of the exchange product (test infrastructure only).

The Coulomb matrix is Hermitian positive definite (it is the Gram matrix of the
Coulomb kernel on the biorthogonal functions, eq. "coulomb matrix"), so
v = L L^H with L lower triangular and a positive real diagonal, and

    A^H v A = (L^H A)^H (L^H A) = Y^H Y,   Y = L^H A.

The oracle uses ``numpy.linalg.cholesky`` on the dense v (a library routine as
a step) -- no blocking beyond what the definition states.
"""
from __future__ import annotations

import numpy as np


def cholesky(v: np.ndarray) -> np.ndarray:
    """Lower L with v = L L^H (NumPy/LAPACK)."""
    return np.linalg.cholesky(v)


def vx_k_cholesky(m_blocks, v_list, w_q) -> np.ndarray:
    """V(k) = -sum_q w_q sum_{n''} Y^H Y with Y = L(q)^H A_{n''}."""
    nb = m_blocks[0].shape[1]
    V = np.zeros((nb, nb), dtype=np.complex128)
    for q, mq in enumerate(m_blocks):
        L = cholesky(v_list[q])
        for npp in range(mq.shape[0]):
            Y = L.conj().T @ mq[npp].T
            V -= w_q[q] * (Y.conj().T @ Y)
    return V
