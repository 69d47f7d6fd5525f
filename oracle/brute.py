"""Brute-force exchange matrix: the literal nested sum (test infrastructure only).

Writes out eq. "vec-mat-vec" (Sec. III.C) term by term in pure Python:

    V_{nn'}(k) = - sum_q w_q sum_{n''} sum_I sum_J conj(M[q][n''][n][I]) v[q][I][J] M[q][n''][n'][J]

For N_MB <= 12, n_b <= 4, n_occ <= 2, N_q <= 3 only.
"""
from __future__ import annotations

import numpy as np


def brute_vx(m_blocks, v_list, w_q) -> np.ndarray:
    nb = len(m_blocks[0][0])
    V = [[0j for _ in range(nb)] for _ in range(nb)]
    for q in range(len(m_blocks)):
        m = m_blocks[q]
        v = v_list[q]
        nmb = len(v)
        for npp in range(len(m)):
            for n in range(nb):
                for n2 in range(nb):
                    s = 0j
                    for i in range(nmb):
                        bra = complex(m[npp][n][i]).conjugate()
                        for j in range(nmb):
                            s += bra * complex(v[i][j]) * complex(m[npp][n2][j])
                    V[n][n2] -= float(w_q[q]) * s
    return np.array(V, dtype=np.complex128)
