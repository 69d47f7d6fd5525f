"""Oracle: the exchange matrix V^x(k) from its definition (test infrastructure only).

Definition (Sec. III.C, eq. "vec-mat-vec"):

    V_{nn'}(k) = - sum_q w_q sum_{n'' occ} sum_{IJ} conj(M^{n n''}_I(k,q)) v_IJ(q) M^{n' n''}_J(k,q)

where M^{n n''}_I(k,q) is the MPB projection of the wavefunction product
(M_I^q phi_{n'' k-q} | phi_{n k}) and v(q) the Coulomb matrix of the MPB
(eq. "coulomb matrix"). The q sum is the Brillouin-zone integration on the mesh
(Sec. II, the sentence following eq. "HF exchange energy"), i.e. a weighted sum
with weights w_q (1/N_q on an equidistant mesh).

Readings taken here where the paper leaves a choice:
  * conjugation: the bra-side projection is conjugated, so with
    A_{n''} = M(k,q)[n''] viewed as an N_MB x n_b matrix, V = -sum w_q A^H v A;
  * the occupied set is the same n_occ bands at every k-q, unit occupation per
    spin channel, one spin channel;
  * the band cutoff n_max (Sec. III) is the column count n_b(k) of M.

Layout of the inputs: ``M`` for one (k,q) is [n_occ][n_b][N_MB] (I fastest).
The Coulomb matrix is given in the paper's transformed MPB order (Fig. 1):
multipole-free MT functions grouped by channel, then one multipole function per
channel, then plane waves; ``assemble_v`` writes it out densely.
"""
from __future__ import annotations

import numpy as np

__all__ = ["assemble_v", "vx_k", "vx_all", "energy_trace", "energy_direct",
           "default_rho", "hermitian_part"]


def assemble_v(E_q: np.ndarray, D: list, C: list) -> np.ndarray:
    """Dense v(q) from the sparse block form (Sec. III.C and the Fig. 1 caption).

    Index order: [mu=0 functions of channel 0, channel 1, ...] (N_s rows), then
    the dense block [multipole function of channel 0..N_ch-1, plane waves].
      v[s_c, s_c]        = D_c        (onsite block of the multipole-free functions)
      v[s_c, N_s + c]    = C_c        (coupling to the channel's own multipole function)
      v[N_s + c, s_c]    = C_c^H
      v[N_s:, N_s:]      = E(q)
    Every other element is zero.
    """
    sizes = [d.shape[0] for d in D]
    n_s = int(sum(sizes))
    n_d = E_q.shape[0]
    n = n_s + n_d
    v = np.zeros((n, n), dtype=np.complex128)
    off = 0
    for c, (d, cv) in enumerate(zip(D, C)):
        b = d.shape[0]
        if b:
            v[off:off + b, off:off + b] = d
            v[off:off + b, n_s + c] = cv
            v[n_s + c, off:off + b] = cv.conj()
        off += b
    v[n_s:, n_s:] = E_q
    return v


def vx_k(m_blocks, v_list, w_q) -> np.ndarray:
    """V^x(k) for one k.

    m_blocks[q] : complex array [n_occ][n_b][N_MB(q)]
    v_list[q]   : dense Hermitian v(q), N_MB(q) x N_MB(q)
    w_q         : q weights
    Returns the raw n_b x n_b complex128 matrix (no symmetrisation).
    """
    nb = m_blocks[0].shape[1]
    V = np.zeros((nb, nb), dtype=np.complex128)
    for q, mq in enumerate(m_blocks):
        v = v_list[q]
        for npp in range(mq.shape[0]):
            A = mq[npp].T                      # N_MB x n_b, column n = M^{n n''}
            V -= w_q[q] * (A.conj().T @ (v @ A))
    return V


def vx_all(cfg, m_of_kq, v_list):
    """V^x(k) for every irreducible k; ``m_of_kq(k, q)`` returns M(k,q)."""
    w = cfg.weights_q()
    return [vx_k([m_of_kq(k, q) for q in range(cfg.n_q)], v_list, w) for k in range(cfg.n_k)]


def hermitian_part(V: np.ndarray) -> np.ndarray:
    return 0.5 * (V + V.conj().T)


def default_rho(n_b: int, n_occ: int) -> np.ndarray:
    """Spin-degenerate density matrix in the band basis: 2 on occupied bands."""
    r = np.zeros((n_b, n_b), dtype=np.complex128)
    r[np.arange(n_occ), np.arange(n_occ)] = 2.0
    return r


def energy_trace(V_list, w_k, rho_list) -> float:
    """E_x = 1/2 sum_k w_k Tr(rho_k V_k).

    Follows eq. "HF exchange energy" (the -1/2 sum over spins and occupied pairs)
    together with eq. "x-potential(wf)": with spin degeneracy the spin sum gives
    a factor 2 absorbed in rho = 2 P_occ.
    """
    e = 0.0
    for V, w, rho in zip(V_list, w_k, rho_list):
        e += w * np.trace(rho @ V).real
    return 0.5 * e


def energy_direct(cfg, m_of_kq, v_list) -> float:
    """E_x summed directly as quadratic forms, never forming V.

    E = - sum_k w_k sum_q w_q sum_{n<n_occ} sum_{n''<n_occ} a^H v(q) a,
    a = M^{n n''}(k,q); the spin sum (x2) cancels the 1/2 of the energy.
    """
    wq, wk = cfg.weights_q(), cfg.weights_k()
    e = 0.0
    for k in range(cfg.n_k):
        for q in range(cfg.n_q):
            mq = m_of_kq(k, q)
            v = v_list[q]
            for npp in range(cfg.n_occ):
                for n in range(cfg.n_occ):
                    a = mq[npp, n]
                    e -= wk[k] * wq[q] * np.vdot(a, v @ a).real
    return e
