"""Back-transform of the exchange matrix to the LAPW basis (test infrastructure only).

Sec. III.A, eq. "APW trafo": V^x in the basis functions G is the band-space V^x
multiplied on the left by the inverse of the eigenvector matrix's adjoint and on
the right by the inverse of the eigenvectors. With generalized orthonormal
eigenvectors (c^H S c = 1) that inverse is c^H S, so

    V_GG' = sum_{n n'} Z_{G n} V_{n n'} conj(Z_{G' n'}),   Z = S c,

i.e. V_GG = Z V Z^H. (The printed left factor carries S* with the indices of S;
for the Hermitian overlap the adjoint's elements are meant, which makes V_GG
Hermitian; for a real S, as with inversion symmetry, both readings coincide.)
"""
from __future__ import annotations

import numpy as np


def back_transform(Z: np.ndarray, V: np.ndarray) -> np.ndarray:
    """V_GG = Z V Z^H (two library matrix products)."""
    Z = np.asarray(Z, dtype=np.complex128)
    return Z @ np.asarray(V, dtype=np.complex128) @ Z.conj().T


def back_transform_loops(Z: np.ndarray, V: np.ndarray) -> np.ndarray:
    """The same sum written out element by element (tiny sizes only)."""
    nG, nb = Z.shape
    out = np.zeros((nG, nG), dtype=np.complex128)
    for g in range(nG):
        for h in range(nG):
            s = 0j
            for n in range(nb):
                for m in range(nb):
                    s += Z[g, n] * V[n, m] * np.conj(Z[h, m])
            out[g, h] = s
    return out
