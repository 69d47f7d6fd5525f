"""Input-rounding emulation of the reduced-precision product modes (test only).

Predicts the error a kernel running the Cholesky/HERK form in a reduced product
precision should show against the float64 oracle, so that a GPU parity test can
demand "within a small factor of the predicted error" instead of an arbitrary
tolerance. Modelled: rounding of the operands to the mode's storage, products
of split pieces (exact in binary32, as on the matrix cores), accumulation in
binary32 (NumPy float32 / complex64 GEMMs; the summation order differs from the
hardware's but the error magnitude does not), rounding of Y = L^H A to binary32,
and the float64 diagonal and q sum.

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


def _prod_bf16x6(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Complex a @ b with each real product done with the six leading split terms."""
    def mm(x, y):
        xh, xm, xl = split3_bf16(x)
        yh, ym, yl = split3_bf16(y)
        return xh @ yh + xh @ ym + xm @ yh + xh @ yl + xm @ ym + xl @ yh

    re = mm(a.real, b.real) - mm(a.imag, b.imag)
    im = mm(a.real, b.imag) + mm(a.imag, b.real)
    return re + 1j * im


def _prod_bf16x3(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Complex a @ b with each real product done as hi*hi + hi*lo + lo*hi."""
    ar_h, ar_l = split_bf16(a.real)
    ai_h, ai_l = split_bf16(a.imag)
    br_h, br_l = split_bf16(b.real)
    bi_h, bi_l = split_bf16(b.imag)

    def mm(xh, xl, yh, yl):
        return xh @ yh + xh @ yl + xl @ yh

    re = mm(ar_h, ar_l, br_h, br_l) - mm(ai_h, ai_l, bi_h, bi_l)
    im = mm(ar_h, ar_l, bi_h, bi_l) + mm(ai_h, ai_l, br_h, br_l)
    return re + 1j * im


def _pieces(x: np.ndarray, n: int):
    return split_bf16(x) if n == 2 else split3_bf16(x)


_PAIRS = {2: ((0, 0), (0, 1), (1, 0)), 3: ((0, 0), (0, 1), (1, 0), (0, 2), (1, 1), (2, 0))}


def _real_split_mm32(x: np.ndarray, y: np.ndarray, n: int) -> np.ndarray:
    """sum over leading piece pairs of x_i @ y_j, each GEMM accumulated in float32."""
    px = [p.astype(np.float32) for p in _pieces(x, n)]
    py = [p.astype(np.float32) for p in _pieces(y, n)]
    acc = np.zeros((x.shape[0], y.shape[1]), dtype=np.float32)
    for i, j in _PAIRS[n]:
        acc = acc + px[i] @ py[j]
    return acc.astype(np.float64)


def _prod_split32(a: np.ndarray, b: np.ndarray, n: int) -> np.ndarray:
    """Complex a @ b as four real split products with float32 accumulation."""
    re = _real_split_mm32(a.real, b.real, n) - _real_split_mm32(a.imag, b.imag, n)
    im = _real_split_mm32(a.real, b.imag, n) + _real_split_mm32(a.imag, b.real, n)
    return re + 1j * im


def vx_k_emulated(m_blocks, L_list, w_q, mode: str) -> np.ndarray:
    """Emulated HERK-form V(k) for ``mode`` in {"fp64", "fp32", "bf16x3", "bf16x6"}.

    L_list[q] is the float64 Cholesky factor of the dense v(q).
    """
    nb = m_blocks[0].shape[1]
    V = np.zeros((nb, nb), dtype=np.complex128)
    for q, mq in enumerate(m_blocks):
        Uh = L_list[q].conj().T
        for npp in range(mq.shape[0]):
            A = mq[npp].T
            if mode == "fp64":
                Y = Uh @ A
                P = Y.conj().T @ Y
            elif mode == "fp32":
                Y = (Uh.astype(np.complex64) @ A.astype(np.complex64)).astype(np.complex128)
                Y32 = Y.astype(np.complex64)
                P = (Y32.conj().T @ Y32).astype(np.complex128)
            elif mode == "bf16x3":
                Y = round_fp32(_prod_split32(Uh, A, 2))
                P = _prod_split32(Y.conj().T, Y, 2)
            elif mode == "bf16x6":
                Y = round_fp32(_prod_split32(Uh, A, 3))
                P = _prod_split32(Y.conj().T, Y, 3)
            else:
                raise ValueError(mode)
            d = np.sum(np.abs(Y) ** 2, axis=0)      # diagonal in float64 from the mode's Y
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
