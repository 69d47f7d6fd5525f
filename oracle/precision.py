"""Input-rounding emulation of the reduced-precision product modes (test only).

Predicts the error a kernel running the Cholesky/HERK form in a reduced product
precision should show against the float64 oracle, so that a GPU parity test can
demand "within a small factor of the predicted error" instead of an arbitrary
tolerance. Modelled: rounding of the operands to the mode's storage, products
of split pieces (exact in binary32, as on the matrix cores), accumulation in
binary32 sequentially over the contraction index in chunks of one matrix-core
instruction's K (4 for fp32, 32 for the bf16 modes), the real and imaginary
products of a chunk added in turn, as the kernels accumulate (a single blocked
float32 GEMM would understate the growth of the rounding error with K),
rounding of Y = L^H A to binary32, and the float64 diagonal and q sum.

Modes
  fp32   -- operands rounded to IEEE binary32 (round to nearest even).
  bf16x3 -- x ~ hi + lo with hi = bf16(x), lo = bf16(x - hi) (round to nearest
            even, 8 significant bits), product hi*hi + hi*lo + lo*hi
            (Henry, Tang & Heinecke, ARITH 2019: the lo*lo term is dropped).
  bf16x6 -- three-way split x ~ hi + mid + lo (24 significant bits), product
            hh + hm + mh + hl + mm + lh (the same paper's six-product variant).
The diagonal V_nn is formed from the mode's Y in float64 and the q sum is float64.
"""
from __future__ import annotations

import numpy as np


def round_fp32(x: np.ndarray) -> np.ndarray:
    if np.iscomplexobj(x):
        return x.astype(np.complex64).astype(np.complex128)
    return x.astype(np.float32).astype(np.float64)


def bf16_rne(x: np.ndarray) -> np.ndarray:
    """Round float64 values to 8 significant bits, ties to even."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)                 # x = m 2^e, 0.5 <= |m| < 1
    r = np.rint(m * 256.0) / 256.0     # np.rint: round half to even
    return np.ldexp(r, e)


def split_bf16(x: np.ndarray):
    """Return (hi, lo) real arrays of the split of a real array."""
    hi = bf16_rne(x)
    lo = bf16_rne(x - hi)
    return hi, lo


def split3_bf16(x: np.ndarray):
    """Return (hi, mid, lo) with each part bf16 (RNE) of the remaining residual."""
    hi = bf16_rne(x)
    mid = bf16_rne(x - hi)
    lo = bf16_rne(x - hi - mid)
    return hi, mid, lo


def _pieces(x: np.ndarray, n: int):
    return split_bf16(x) if n == 2 else split3_bf16(x)


_PAIRS = {2: ((0, 0), (0, 1), (1, 0)), 3: ((0, 0), (0, 1), (1, 0), (0, 2), (1, 1), (2, 0))}


def _cmm32_seq(a: np.ndarray, b: np.ndarray, n: int, chunk: int) -> np.ndarray:
    """Complex a @ b in binary32: K in chunks, each chunk's real products (the sum of
    the leading piece pairs for n = 2, 3; the plain product for n = 1) added to the
    real accumulator (ar br, then -ai bi) and the imaginary one (ar bi, then ai br)."""
    def parts(x):
        if n == 1:
            return [x.astype(np.float32)]
        return [p.astype(np.float32) for p in _pieces(x, n)]
    pairs = ((0, 0),) if n == 1 else _PAIRS[n]
    ar, ai = parts(a.real), parts(-a.imag)
    ai_pos = parts(a.imag)
    br, bi = parts(b.real), parts(b.imag)
    acc_r = np.zeros((a.shape[0], b.shape[1]), dtype=np.float32)
    acc_i = np.zeros_like(acc_r)

    def chunk_mm(x, y, k0, k1):
        t = np.zeros_like(acc_r)
        for i, j in pairs:
            t = t + x[i][:, k0:k1] @ y[j][k0:k1, :]
        return t

    for k0 in range(0, a.shape[1], chunk):
        k1 = min(k0 + chunk, a.shape[1])
        acc_r = acc_r + chunk_mm(ar, br, k0, k1)
        acc_r = acc_r + chunk_mm(ai, bi, k0, k1)
        acc_i = acc_i + chunk_mm(ar, bi, k0, k1)
        acc_i = acc_i + chunk_mm(ai_pos, br, k0, k1)
    return acc_r.astype(np.float64) + 1j * acc_i.astype(np.float64)


_MODE_PIECES = {"fp32": (1, 4), "bf16x3": (2, 32), "bf16x6": (3, 32)}


def vx_k_emulated(m_blocks, L_list, w_q, mode: str) -> np.ndarray:
    """Emulated HERK-form V(k) for ``mode`` in {"fp64", "fp32", "bf16x3", "bf16x6"}.

    L_list[q] is the float64 Cholesky factor of the dense v(q).
    """
    nb = m_blocks[0].shape[1]
    V = np.zeros((nb, nb), dtype=np.complex128)
    for q, mq in enumerate(m_blocks):
        Uh = L_list[q].conj().T
        # Y = L^H A for every n'' at once: the columns of a product are independent, so
        # one product over [A_0 | A_1 | ...] gives each n'' its own Y
        A = np.concatenate([mq[npp].T for npp in range(mq.shape[0])], axis=1)
        if mode == "fp64":
            Y = Uh @ A
        elif mode in _MODE_PIECES:
            n, ch = _MODE_PIECES[mode]
            Y = round_fp32(_cmm32_seq(Uh, A, n, ch))
        else:
            raise ValueError(mode)
        for npp in range(mq.shape[0]):
            Yn = Y[:, npp * nb:(npp + 1) * nb]
            if mode == "fp64":
                P = Yn.conj().T @ Yn
            else:
                n, ch = _MODE_PIECES[mode]
                P = _cmm32_seq(Yn.conj().T, Yn, n, ch)
            d = np.sum(np.abs(Yn) ** 2, axis=0)     # diagonal in float64 from the mode's Y
            P[np.arange(nb), np.arange(nb)] = d
            V -= w_q[q] * P
    return V


def normalised_eig_error(V: np.ndarray, V_ref: np.ndarray, rho_max: float) -> float:
    """max_i |lambda_i - lambda_i^ref| / rho_max (eigenvalues of the Hermitian parts)."""
    a = np.linalg.eigvalsh(0.5 * (V + V.conj().T))
    b = np.linalg.eigvalsh(0.5 * (V_ref + V_ref.conj().T))
    return float(np.max(np.abs(a - b)) / rho_max)


def normwise_error(V: np.ndarray, V_ref: np.ndarray) -> float:
    """max_ij |V - V_ref| / max_ij |V_ref|."""
    return float(np.max(np.abs(V - V_ref)) / np.max(np.abs(V_ref)))
