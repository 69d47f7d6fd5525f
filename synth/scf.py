"""Synthetic outer self-consistency iterations for the learned V^x extrapolator.

Stand-in for the outer loop of the nested scheme (Sec. IV): the occupied
subspace of every k' drifts from step to step, with a rank-4 perturbation whose
amplitude halves each step, and the product-basis projections follow it.

* U_1(k') = the first n_occ columns of the n_b x n_b identity (reference
  occupied bands).
* U_{t+1}(k') = orthonormal basis (QR) of U_t(k') + a_t X(k') diag(c_t) Y(k')^H,
  a_t = a0 * 0.5^(t-1); X(k') (n_b x 4) and Y(k') (n_occ x 4) are fixed complex
  Gaussian matrices per k' with unit columns (the modes the density moves
  along), c_t (4 reals, shared by all k') are fresh Gaussian coefficients per
  step.
* P_t(k') = U_t U_t^H, the density matrix in the reference-band basis.
* M_t(k, q) = M_ref(k, q) mixed over its reference-band index n'' with conj(U_t(k'))
  for k' = (k + q) mod n_k (the synthetic meshes carry no symmetry map, so each
  (k, q) is assigned an irreducible k - q by this rule). M_ref(k, q) has n_b
  reference bands in n''; its first n_occ slices are the workload's own M(k, q).

V^x is then exactly linear in P_t for fixed M_ref and v (a mixed sum over n''
becomes a sum weighted by P_t).
"""
from __future__ import annotations

import dataclasses
from typing import List

import numpy as np

from . import Config, normal_pairs, sm_int, m_block

RANK = 4
TAG_SCF = 0x5CF


def k_prime(cfg: Config, k: int, q: int) -> int:
    return (k + q) % cfg.n_k


def _gauss_c(seed: int, shape) -> np.ndarray:
    n = int(np.prod(shape))
    z0, z1 = normal_pairs(seed, 0, n)
    return ((z0 + 1j * z1) / np.sqrt(2.0)).reshape(shape)


def occupied_sequence(cfg: Config, n_iter: int, a0: float = 0.1, seed: int = 0) -> List[List[np.ndarray]]:
    """U_t(k') for t = 1..n_iter: list over t of lists over k' of n_b x n_occ complex arrays."""
    nb = cfg.n_bands[0]
    if any(b != nb for b in cfg.n_bands):
        raise ValueError("the synthetic outer iterations assume one band count for all k")
    base = sm_int(sm_int(cfg.seed + seed, cfg.tag), TAG_SCF)
    unit = lambda A: A / np.linalg.norm(A, axis=0)
    X = [unit(_gauss_c(sm_int(base, 2 * kp), (nb, RANK))) for kp in range(cfg.n_k)]
    Y = [unit(_gauss_c(sm_int(base, 2 * kp + 1), (cfg.n_occ, RANK))) for kp in range(cfg.n_k)]
    U = [np.eye(nb, cfg.n_occ, dtype=np.complex128) for _ in range(cfg.n_k)]
    seq = [[u.copy() for u in U]]
    for t in range(1, n_iter):
        a = a0 * 0.5 ** (t - 1)
        c0, _ = normal_pairs(sm_int(base, 1000003 + t), 0, RANK)
        for kp in range(cfg.n_k):
            Q, R = np.linalg.qr(U[kp] + a * (X[kp] * c0) @ Y[kp].conj().T)
            U[kp] = Q * np.sign(np.real(np.diag(R)))          # fixed column phases (P does not depend on them)
        seq.append([u.copy() for u in U])
    return seq


def density(U: List[np.ndarray]) -> List[np.ndarray]:
    return [u @ u.conj().T for u in U]


def density_vector(P: List[np.ndarray]) -> np.ndarray:
    """P of every k' as one real float64 vector: k' outer, column-major, (Re, Im) interleaved."""
    out = []
    for M in P:
        cm = np.asarray(M, dtype=np.complex128).T.ravel()
        out.append(np.stack([cm.real, cm.imag], axis=1).ravel())
    return np.concatenate(out)


def reference_config(cfg: Config) -> Config:
    """The workload with n_b reference bands in the n'' slot of M."""
    return dataclasses.replace(cfg, n_occ=cfg.n_bands[0])


def m_ref_block(cfg: Config, k: int, q: int) -> np.ndarray:
    """M_ref(k, q) as [n_b (reference n'')][n_b][N_MB]."""
    return m_block(reference_config(cfg), k, q)


def mix(m_ref: np.ndarray, U: np.ndarray) -> np.ndarray:
    """M(k,q)[j] = sum_m conj(U[m, j]) M_ref(k,q)[m]: [n_occ][n_b][N_MB]."""
    nref = m_ref.shape[0]
    return (U.conj().T @ m_ref.reshape(nref, -1)).reshape((U.shape[1],) + m_ref.shape[1:])


def make_feed(cfg: Config, n_iter: int, device, a0: float = 0.1, seed: int = 0):
    """feed(t) -> (M_t per k as flat complex128 device tensors, P_t as a float64 device vector).

    M_ref is generated once on the host and the mixing runs on the host (sizes of
    the test workloads)."""
    import torch

    Us = occupied_sequence(cfg, n_iter, a0=a0, seed=seed)
    mref = {(k, q): m_ref_block(cfg, k, q) for k in range(cfg.n_k) for q in range(cfg.n_q)}

    def feed(t: int):
        U = Us[t - 1]
        Ms = [torch.from_numpy(np.concatenate([mix(mref[k, q], U[k_prime(cfg, k, q)]).ravel()
                                               for q in range(cfg.n_q)])).to(device)
              for k in range(cfg.n_k)]
        P = torch.from_numpy(density_vector(density(U))).to(device)
        return Ms, P

    return feed


def make_feed_device(cfg: Config, n_iter: int, device, a0: float = 0.1, seed: int = 0, dtype: str = "c64"):
    """``make_feed`` for whole workloads: M_ref drawn on the GPU by the seeded generator
    (the reference configuration's blocks, n_b reference bands in n''), and M_t(k, q) =
    U_t(k')^H M_ref(k, q) formed on the GPU per pair into buffers reused across the
    iterations (a complex product of (n_occ x n_b) by (n_b x n_b N_MB)). Returns feed(t) as
    ``make_feed`` does; the M_t tensors of one call are overwritten by the next."""
    import torch

    from . import m_all_device

    dev = torch.device(device)
    tdt = torch.complex64 if dtype == "c64" else torch.complex128
    Us = occupied_sequence(cfg, n_iter, a0=a0, seed=seed)
    rcfg = reference_config(cfg)
    nb, no = cfg.n_bands[0], cfg.n_occ
    mref = [m_all_device(rcfg, k, dtype, dev) for k in range(cfg.n_k)]
    outs = [torch.empty(sum(no * nb * cfg.n_mb(q) for q in range(cfg.n_q)), dtype=tdt, device=dev)
            for _ in range(cfg.n_k)]

    def feed(t: int):
        U = Us[t - 1]
        Uh = [torch.from_numpy(np.ascontiguousarray(u.conj().T)).to(dev, tdt) for u in U]
        for k in range(cfg.n_k):
            o_ref = o_out = 0
            for q in range(cfg.n_q):
                nmb = cfg.n_mb(q)
                src = mref[k][o_ref:o_ref + nb * nb * nmb].view(nb, nb * nmb)
                dst = outs[k][o_out:o_out + no * nb * nmb].view(no, nb * nmb)
                torch.matmul(Uh[k_prime(cfg, k, q)], src, out=dst)
                o_ref += nb * nb * nmb
                o_out += no * nb * nmb
        P = torch.from_numpy(density_vector(density(U))).to(dev)
        return outs, P

    return feed
