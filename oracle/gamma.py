"""Gamma-point term of the exchange matrix (test infrastructure only).

The Coulomb matrix diverges like 1/q^2 at q = 0 (Sec. III.E, "Singularity of the
Coulomb matrix"). Its divergent part, taken in the plane-wave representation
exp(iq.r) and with the overlaps reduced to Kronecker deltas near q = 0, adds to
the occupied diagonal of V^x a term that is integrated analytically once 1/q^2
is damped by exp(-beta q^2) (the function of eq. "F(q)"), minus the part of that
integral the q-mesh sum already holds (the double-counting term of
eq. "divergence"). With a cutoff q0 fixed by exp(-beta q0^2) = beta the result
is eq. "div final":

    V_nn'|div = -delta_nn' f_n C,
    C = erf(sqrt(beta) q0) / sqrt(pi beta)
        - 4 pi / (N Omega) * sum_{p, 0 < |p| <= q0} exp(-beta |p|^2) / |p|^2,

where p runs over all points q + G of the q mesh (every G), N is the number of
mesh points and Omega the unit-cell volume. The factor 4 pi in front of the sum
is this oracle's reading of the printed 1/(N Omega): (1/(N Omega)) sum over the
mesh is the Riemann sum of (2 pi)^-3 times the integral, and the first term is
(1/(2 pi^2)) = 4 pi (2 pi)^-3 times the same integral, so only 4 pi / (N Omega)
makes the bracket vanish as the mesh is refined.

The lattice sum enumerates every integer triple j of a box that contains the
sphere |p| <= q0 and keeps the points inside it: plain, slow and exhaustive.
"""
from __future__ import annotations

import math

import numpy as np


def q0_of_beta(beta: float) -> float:
    """Cutoff with exp(-beta q0^2) = beta (Sec. III.E, after eq. "div final")."""
    if not 0.0 < beta < 1.0:
        raise ValueError("beta must lie in (0, 1)")
    return math.sqrt(-math.log(beta) / beta)


def integral_term(beta: float, q0: float) -> float:
    """(1/(2 pi^2)) * integral over |q| <= q0 of exp(-beta q^2)/q^2 d^3q.

    In spherical coordinates the q^2 of the volume element cancels the 1/q^2:
    (4 pi / (2 pi^2)) * int_0^q0 exp(-beta q^2) dq = erf(sqrt(beta) q0) / sqrt(pi beta).
    """
    return math.erf(math.sqrt(beta) * q0) / math.sqrt(math.pi * beta)


def cell_volume(recip: np.ndarray) -> float:
    """Omega = (2 pi)^3 / |det B| for reciprocal vectors in the rows of B."""
    return (2.0 * math.pi) ** 3 / abs(float(np.linalg.det(recip)))


def box_bounds(recip: np.ndarray, mesh, q0: float) -> np.ndarray:
    """Largest |j_i| of a point sum_i (j_i / mesh_i) b_i with |p| <= q0.

    With real-space vectors a_i (a_i . b_j = 2 pi delta_ij), j_i / mesh_i = p . a_i / (2 pi),
    so |j_i| <= mesh_i q0 |a_i| / (2 pi).
    """
    a = 2.0 * math.pi * np.linalg.inv(recip).T
    return np.floor(np.asarray(mesh) * q0 * np.linalg.norm(a, axis=1) / (2.0 * math.pi)).astype(np.int64)


def lattice_sum(recip: np.ndarray, mesh, beta: float, q0: float | None = None) -> tuple[float, int]:
    """sum over mesh points p = sum_i (j_i/mesh_i) b_i with 0 < |p| <= q0 of exp(-beta p^2)/p^2.

    Returns (sum, number of terms). One j_0 plane at a time; numpy's pairwise sum inside a plane.
    """
    if q0 is None:
        q0 = q0_of_beta(beta)
    g = np.asarray(recip, dtype=np.float64) / np.asarray(mesh, dtype=np.float64)[:, None]
    J = box_bounds(recip, mesh, q0)
    j1 = np.arange(-J[1], J[1] + 1, dtype=np.float64)
    j2 = np.arange(-J[2], J[2] + 1, dtype=np.float64)
    J1, J2 = np.meshgrid(j1, j2, indexing="ij")
    total, count = 0.0, 0
    for j0 in range(-int(J[0]), int(J[0]) + 1):
        p = j0 * g[0][None, None, :] + J1[..., None] * g[1] + J2[..., None] * g[2]
        p2 = np.sum(p * p, axis=-1)
        keep = (p2 > 0.0) & (p2 <= q0 * q0)
        x = p2[keep]
        total += float(np.sum(np.exp(-beta * x) / x))
        count += int(x.size)
    return total, count


def gamma_term(recip: np.ndarray, mesh, beta: float) -> float:
    """C of eq. "div final" (with the 4 pi reading of its prefactor)."""
    q0 = q0_of_beta(beta)
    s, _ = lattice_sum(recip, mesh, beta, q0)
    n = int(np.prod(mesh))
    return integral_term(beta, q0) - 4.0 * math.pi / (n * cell_volume(recip)) * s


def apply_gamma(V: np.ndarray, n_occ: int, C: float) -> np.ndarray:
    """V + V|div: subtract C from V_nn for the occupied bands (occupation 1 per spin)."""
    out = np.array(V, dtype=np.complex128, copy=True)
    for n in range(min(n_occ, out.shape[0])):
        out[n, n] -= C
    return out
