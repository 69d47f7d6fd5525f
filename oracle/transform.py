"""Multipole-moment rotation of the MT functions (test infrastructure only).

Sec. III.C ("Sparsity of the Coulomb matrix"): within one atom and LM channel,
the radial MT functions M_{aLP}(r) have multipole moments
mu_{aLP} = int_0^S M_{aLP}(r) r^{L+2} dr. A real orthogonal change of basis of
the functions of a channel can leave only one function with a nonzero moment;
the others are multipole-free and produce no field outside their sphere, which
is what makes the Coulomb matrix block-sparse.

The paper writes the two-function case explicitly; for n functions it only says
that the procedure generalises. Reading used here: a Householder reflector
H = I - 2 u u^T / (u^T u), u = mu - |mu| e_m, which maps mu to |mu| e_m, so the
new function m carries the whole moment and all others have zero moment.
For n = 2 this coincides with the paper's formula up to the sign of the
multipole-free function.

A change of basis M'_i = sum_j U_ij M_j (U real orthogonal) transforms the
vectors as m' = U m and the Coulomb matrix as v' = U v U^T, so that
m'^H v' m' = m^H v m: the exchange matrix is invariant.
"""
from __future__ import annotations

import numpy as np


def two_function_rotation(mu1: float, mu2: float) -> np.ndarray:
    """The paper's 2x2 transformation: rows give (M'_1, M'_2) in terms of (M_1, M_2).

    M'_1 = (mu1 M1 + mu2 M2)/|mu| carries the moment, M'_2 = (mu2 M1 - mu1 M2)/|mu|
    is multipole-free.
    """
    r = np.hypot(mu1, mu2)
    return np.array([[mu1, mu2], [mu2, -mu1]]) / r


def householder_rotation(mu: np.ndarray, m: int) -> np.ndarray:
    """Real orthogonal U with U @ mu = |mu| e_m (rows = new functions)."""
    mu = np.asarray(mu, dtype=np.float64)
    n = mu.shape[0]
    e = np.zeros(n)
    e[m] = 1.0
    u = mu - np.linalg.norm(mu) * e
    nu = u @ u
    if nu < 1e-300:               # mu already along e_m
        return np.eye(n)
    return np.eye(n) - 2.0 * np.outer(u, u) / nu


def moments(U: np.ndarray, mu: np.ndarray) -> np.ndarray:
    """Multipole moments of the transformed functions: (U mu)_i."""
    return U @ mu


def sparse_order_unitary(ch_nrad, mu_list, n_d: int) -> np.ndarray:
    """Orthogonal matrix taking an untransformed MPB to the sparse order.

    Untransformed order: channel by channel, each channel's nrad_c functions
    contiguous, then the plane waves. Sparse (Fig. 1) order: all multipole-free
    functions (channel by channel), then one multipole function per channel,
    then the plane waves. Returns T with m_sparse = T m_orig, v_sparse = T v_orig T^T.
    """
    n_ch = len(ch_nrad)
    n_s = int(sum(b - 1 for b in ch_nrad))
    n_mt = int(sum(ch_nrad))
    n_pw = n_d - n_ch
    n = n_mt + n_pw
    T = np.zeros((n, n))
    orig = 0
    s_off = 0
    for c, b in enumerate(ch_nrad):
        Uc = householder_rotation(mu_list[c], b - 1)   # last local function carries mu
        # local rows 0..b-2 -> multipole-free slots; row b-1 -> multipole slot
        for i in range(b - 1):
            T[s_off + i, orig:orig + b] = Uc[i]
        T[n_s + c, orig:orig + b] = Uc[b - 1]
        orig += b
        s_off += b - 1
    for p in range(n_pw):
        T[n_s + n_ch + p, n_mt + p] = 1.0
    return T
