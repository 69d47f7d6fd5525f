"""Float64 reference of the learned extrapolator's encoding -- TEST INFRASTRUCTURE ONLY.

Between exact evaluations of V^x (Sec. III.C) the extension predicts the change
of V^x(k) caused by a change of the density matrix. V^x is linear in the
density matrix for fixed product-basis projections, so the map to learn is
dV = L(dP). The network sees a fixed-size encoding of dP and returns a
fixed-size encoding of dV(k) for every k (the blocks of all k concatenated):

* input  x = S vec(dP) / |vec(dP)|  (m entries),
  where vec(dP) stacks, for every k' and column j and row i, Re then Im of
  dP_k'[i, j] (columns of n_b x n_b complex matrices, k' outermost), and S is
  the m x D Rademacher sketch S_ij = +-1/sqrt(m), the sign taken from the top
  bit of SplitMix64(seed) output number i*D + j (set bit: minus);
* output y(k) = enc(B_k^H dV(k) B_k) / |vec(dP)|, B_k the eigenvectors of the
  anchor V^x(k) for its n_blk most negative eigenvalues; enc writes an n_blk x
  n_blk Hermitian H as the real matrix R (row-major) with R[i, j] = Re H[i, j]
  for i <= j and R[j, i] = Im H[i, j] for i < j.

The prediction is V(k) = V_anchor(k) + |vec(dP)| B_k dec(y(k)) B_k^H: the part
of dV outside span(B_k) is left at the anchor. The judge compares the n_blk
most negative eigenvalues with those of the exact V^x.
"""
from __future__ import annotations

from typing import Sequence

import numpy as np


def dp_vector(dP: Sequence[np.ndarray]) -> np.ndarray:
    """Real vector of the density-matrix change: k' outer, then column, row, (Re, Im)."""
    parts = []
    for M in dP:
        cm = np.asarray(M, dtype=np.complex128).T.ravel()   # column-major order of M
        parts.append(np.stack([cm.real, cm.imag], axis=1).ravel())
    return np.concatenate(parts)


def rademacher_signs(seed: int, rows: int, cols: int, stream) -> np.ndarray:
    """rows x cols matrix of +-1, sign of entry (i, j) from output i*cols + j."""
    x = stream(seed, 0, rows * cols).reshape(rows, cols)
    return np.where((x >> np.uint64(63)) != 0, -1.0, 1.0)


def sketch(v: np.ndarray, m: int, seed: int, stream):
    """(S v / |v|, |v|) with S = rademacher_signs / sqrt(m); a zero v gives zeros."""
    nrm = float(np.linalg.norm(v))
    S = rademacher_signs(seed, m, v.size, stream) / np.sqrt(m)
    if nrm == 0.0:
        return np.zeros(m), 0.0
    return S @ (v / nrm), nrm


def basis(V: np.ndarray, n_blk: int) -> np.ndarray:
    """Eigenvectors of the Hermitian V for its n_blk smallest (most negative) eigenvalues."""
    w, Z = np.linalg.eigh(0.5 * (V + V.conj().T))
    return Z[:, :n_blk]


def encode(Hm: np.ndarray) -> np.ndarray:
    nb = Hm.shape[0]
    R = np.zeros((nb, nb))
    for i in range(nb):
        for j in range(i, nb):
            R[i, j] = Hm[i, j].real
            if i < j:
                R[j, i] = Hm[i, j].imag
    return R.ravel()


def decode(y: np.ndarray, nb: int) -> np.ndarray:
    R = np.asarray(y, dtype=np.float64).reshape(nb, nb)
    Hm = np.zeros((nb, nb), dtype=np.complex128)
    for i in range(nb):
        Hm[i, i] = R[i, i]
        for j in range(i + 1, nb):
            Hm[i, j] = R[i, j] + 1j * R[j, i]
            Hm[j, i] = np.conj(Hm[i, j])
    return Hm


def project(dV: np.ndarray, B: np.ndarray, scale: float) -> np.ndarray:
    """enc(B^H dV B) * scale."""
    return encode(B.conj().T @ dV @ B) * scale


def expand(V_anchor: np.ndarray, B: np.ndarray, y: np.ndarray, scale: float) -> np.ndarray:
    """V_anchor + scale * B dec(y) B^H."""
    return V_anchor + scale * (B @ decode(y, B.shape[1]) @ B.conj().T)


def lowest_eigs(V: np.ndarray, n_blk: int) -> np.ndarray:
    return np.linalg.eigvalsh(0.5 * (V + V.conj().T))[:n_blk]


def judge_error(V_pred: np.ndarray, V_exact: np.ndarray, n_blk: int, rho_max: float) -> float:
    """max |lambda_i(V_pred) - lambda_i(V_exact)| over the n_blk lowest, / rho_max."""
    return float(np.max(np.abs(lowest_eigs(V_pred, n_blk) - lowest_eigs(V_exact, n_blk))) / rho_max)


def ridge_fit(X: np.ndarray, Y: np.ndarray, lam: float) -> np.ndarray:
    """Affine least squares with ridge penalty: returns W (in+1 x out), last row the bias."""
    Xa = np.hstack([X, np.ones((X.shape[0], 1))])
    A = Xa.T @ Xa + lam * np.eye(Xa.shape[1])
    return np.linalg.solve(A, Xa.T @ Y)


def ridge_predict(W: np.ndarray, X: np.ndarray) -> np.ndarray:
    return np.hstack([X, np.ones((X.shape[0], 1))]) @ W
