"""Point-group symmetry of a Gamma-centred q mesh (host-side set-up, no GPU work).

Sec. III.D ("rotate APW" equation): only the operations that leave k invariant
modulo a reciprocal lattice vector (the little group LG(k)) may be used to
reduce the q sum of V^x(k). They split the mesh into orbits; one representative
per orbit forms the extended irreducible wedge EIBZ(k), and a representative q
carries the factor 1/N_{k,q}, N_{k,q} being the number of operations common to
LG(k) and LG(q) (the stabiliser of q inside LG(k)). Rotating the restricted sum
by every operation of LG(k) and adding restores the full sum, since an orbit
has |LG(k)| / N_{k,q} members.

Operations are integer 3x3 matrices R acting on fractional reciprocal
coordinates as row vectors, f -> f R; they are the lattice's point group: the
integer matrices that preserve the reciprocal metric B B^T (entries in
{-1, 0, 1} suffice for the lattices here). Time reversal (k -> -k) adds nothing
for lattices whose point group holds the inversion, as all of these do.
"""
from __future__ import annotations

import itertools
import math

import numpy as np


def point_group(lattice: np.ndarray) -> list:
    """Integer matrices R (acting f -> f R on fractional reciprocal coordinates) that
    preserve the reciprocal metric of the lattice (rows = real-space vectors)."""
    B = 2.0 * math.pi * np.linalg.inv(np.asarray(lattice, dtype=np.float64)).T
    G = B @ B.T
    tol = 1e-9 * float(np.abs(G).max())
    ops = []
    for e in itertools.product((-1, 0, 1), repeat=9):
        R = np.array(e, dtype=np.int64).reshape(3, 3)
        if abs(round(np.linalg.det(R))) != 1:
            continue
        if np.abs(R @ G @ R.T - G).max() <= tol:
            ops.append(R)
    return ops


def _mesh_index(points: np.ndarray):
    """Divisions of the mesh and a map from integer coordinates (mod mesh) to the point index."""
    f = np.asarray(points, dtype=np.float64)
    mesh = np.array([len(np.unique(np.round(np.mod(f[:, i], 1.0), 10))) for i in range(3)], dtype=np.int64)
    key = np.mod(np.rint(f * mesh).astype(np.int64), mesh)
    lut = {tuple(int(x) for x in key[i]): i for i in range(f.shape[0])}
    if len(lut) != f.shape[0] or int(np.prod(mesh)) != f.shape[0]:
        raise ValueError("the points do not form a full Gamma-centred mesh")
    return mesh, key, lut


def _image(key_row, R, mesh, lut):
    img = np.mod(key_row @ R, mesh)
    return lut.get(tuple(int(x) for x in img))


def little_group(k_frac: np.ndarray, ops: list, mesh) -> list:
    """Operations with k R = k modulo a reciprocal lattice vector (k on the mesh)."""
    mesh = np.asarray(mesh, dtype=np.int64)
    kk = np.mod(np.rint(np.asarray(k_frac, dtype=np.float64) * mesh).astype(np.int64), mesh)
    return [R for R in ops if np.array_equal(np.mod(kk @ R, mesh), kk)]


def orbits(points: np.ndarray, ops: list):
    """(representative index of each point, stabiliser size of each point) under ops;
    the representative of an orbit is its smallest index. Operations that map the mesh
    outside itself (none do for a point group of the lattice) raise."""
    mesh, key, lut = _mesh_index(points)
    n = key.shape[0]
    rep = np.full(n, -1, dtype=np.int64)
    stab = np.zeros(n, dtype=np.int64)
    for i in range(n):
        imgs = []
        for R in ops:
            j = _image(key[i], R, mesh, lut)
            if j is None:
                raise ValueError("an operation maps a mesh point off the mesh")
            imgs.append(j)
        rep[i] = min(imgs)
        stab[i] = sum(1 for j in imgs if j == i)
    return rep, stab


def irreducible(points: np.ndarray, ops: list):
    """Irreducible points of the mesh under ops: (indices, weights = orbit size / N)."""
    rep, stab = orbits(points, ops)
    idx = np.unique(rep)
    n = len(points)
    return idx, np.array([len(ops) / stab[i] / n for i in idx])


def eibz_weights(k_frac: np.ndarray, q_points: np.ndarray, ops: list, w_q=None):
    """Pair weights of the EIBZ(k) q sum: w_q / N_{k,q} on the wedge, 0 elsewhere.

    Returns (weights [n_q], |LG(k)|, representative index of every q under LG(k)).
    """
    mesh, _, _ = _mesh_index(q_points)
    lg = little_group(k_frac, ops, mesh)
    rep, stab = orbits(q_points, lg)
    n = len(q_points)
    w_q = np.full(n, 1.0 / n) if w_q is None else np.asarray(w_q, dtype=np.float64)
    w = np.zeros(n)
    for q in range(n):
        if rep[q] == q:
            w[q] = w_q[q] / stab[q]                 # stab[q] = N_{k,q}
    return w, len(lg), rep


def theta_mask(theta: np.ndarray, energies, deg_tol: float = 1e-6, zero_tol: float = 1e-8) -> np.ndarray:
    """Band pairs to compute from the matrix elements of Theta^MT (Sec. III.D, eq. "MT
    stepfuntion"): bands are grouped by degenerate energies (|e_n - e_m| <= deg_tol,
    chained over sorted energies); a pair (n, n') is kept unless the block of theta between
    the group of n and the group of n' is numerically zero (max |.| <= zero_tol times the
    largest |theta|), which marks different irreducible representations."""
    theta = np.asarray(theta)
    e = np.asarray(energies, dtype=np.float64)
    nb = e.size
    order = np.argsort(e, kind="stable")
    group = np.empty(nb, dtype=np.int64)
    g = 0
    for i, n in enumerate(order):
        if i > 0 and e[n] - e[order[i - 1]] > deg_tol:
            g += 1
        group[n] = g
    scale = float(np.abs(theta).max()) if theta.size else 0.0
    ng = g + 1
    nonzero = np.zeros((ng, ng), dtype=bool)
    for a in range(ng):
        ia = np.flatnonzero(group == a)
        for b in range(ng):
            ib = np.flatnonzero(group == b)
            nonzero[a, b] = np.abs(theta[np.ix_(ia, ib)]).max() > zero_tol * scale
    return nonzero[group][:, group]
