"""Pins of the oracle's Gamma-point term (Sec. III.E, eqs. "F(q)", "divergence", "div final").

Each pin comes from outside the oracle's own formula:
  * the cutoff relation exp(-beta q0^2) = beta, as stated after eq. "div final";
  * the analytic integral against numerical quadrature of the radial integral;
  * the lattice sum against brute-force loops over a generous box (tiny sizes),
    and against a unimodular change of the reciprocal basis (the same lattice);
  * the whole bracket against a closed form from lattice-sum theory: on a simple
    cubic mesh of spacing h, integral minus Riemann sum of 1/q^2 approaches
    h * Z, where -Z is the analytically continued cubic-lattice sum
    sum' |n|^-2 over Z^3. Z is evaluated here independently by Ewald's theta-function
    splitting (a textbook formula), so a wrong prefactor, a missing term or a
    dropped lattice point fails this pin;
  * the bracket falls like 1/n as the mesh is refined (the cell around q = 0).
"""
import math

import numpy as np
import pytest
from scipy import integrate
from scipy.special import erfc

import synth
from oracle import gamma as g


def _sc(a):
    return 2.0 * math.pi / a * np.eye(3)


def _cubic_lattice_zeta():
    """Analytic continuation of sum' |n|^-2 over Z^3 by Ewald splitting at s = 1:
    Z = pi * (-3 + sum' [exp(-pi n^2) / (pi n^2) + erfc(sqrt(pi) |n|) / |n|])."""
    r = np.arange(-7, 8)
    X, Y, Z = np.meshgrid(r, r, r, indexing="ij")
    n2 = (X * X + Y * Y + Z * Z).astype(np.float64).ravel()
    n2 = n2[n2 > 0]
    n = np.sqrt(n2)
    return math.pi * (-3.0 + float(np.sum(np.exp(-math.pi * n2) / (math.pi * n2)
                                          + erfc(math.sqrt(math.pi) * n) / n)))


def test_cutoff_relation():
    for beta in (0.005, 0.05, 0.3):
        q0 = g.q0_of_beta(beta)
        assert math.exp(-beta * q0 * q0) == pytest.approx(beta, rel=1e-13)
    with pytest.raises(ValueError):
        g.q0_of_beta(1.0)


def test_integral_term_against_quadrature():
    for beta in (0.005, 0.05, 0.3):
        q0 = g.q0_of_beta(beta)
        # (1/(2 pi^2)) int_{|q| <= q0} exp(-beta q^2) / q^2 d^3q in spherical coordinates
        val, _ = integrate.quad(lambda q: 4.0 * math.pi * q * q * math.exp(-beta * q * q) / (q * q),
                                0.0, q0, epsabs=0.0, epsrel=1e-13, limit=200)
        assert g.integral_term(beta, q0) == pytest.approx(val / (2.0 * math.pi ** 2), rel=1e-11)


def test_lattice_sum_against_brute_force():
    recip = synth.make_config("c2").recip()
    beta = 0.3
    q0 = g.q0_of_beta(beta)
    for mesh in [(1, 1, 1), (2, 3, 1), (3, 3, 3)]:
        gvec = recip / np.asarray(mesh, dtype=np.float64)[:, None]
        s, cnt = 0.0, 0
        R = 14                                   # |j_i| <= 10 holds every point here
        for j0 in range(-R, R + 1):
            for j1 in range(-R, R + 1):
                for j2 in range(-R, R + 1):
                    p = j0 * gvec[0] + j1 * gvec[1] + j2 * gvec[2]
                    p2 = float(p @ p)
                    if 0.0 < p2 <= q0 * q0:
                        s += math.exp(-beta * p2) / p2
                        cnt += 1
        so, co = g.lattice_sum(recip, mesh, beta)
        assert co == cnt
        assert so == pytest.approx(s, rel=1e-12)


def test_lattice_sum_is_basis_independent():
    recip = synth.make_config("c2").recip()
    U = np.array([[1, 1, 0], [0, 1, 0], [2, 0, 1]], dtype=np.float64)    # det 1
    beta = 0.05
    s1, c1 = g.lattice_sum(recip, (3, 3, 3), beta)
    s2, c2 = g.lattice_sum(U @ recip, (3, 3, 3), beta)
    assert c1 == c2
    assert s1 == pytest.approx(s2, rel=1e-12)
    assert g.gamma_term(recip, (3, 3, 3), beta) == pytest.approx(g.gamma_term(U @ recip, (3, 3, 3), beta),
                                                                  abs=1e-12)


def test_bracket_approaches_the_cubic_lattice_constant():
    zeta = _cubic_lattice_zeta()
    assert zeta == pytest.approx(-8.913632917585, abs=1e-9)     # sanity of the Ewald evaluation
    # the paper's beta: the truncation at q0 then costs exp(-beta q0^2)/q0^2 = beta/q0^2 ~ 5e-6 per
    # boundary point, so the limit holds to ~1e-5 already on coarse meshes
    a, beta = 10.0, 0.005
    for n in (2, 3):
        h = 2.0 * math.pi / (a * n)
        C = g.gamma_term(_sc(a), (n, n, n), beta)
        # C = (1/(2 pi^2)) [integral - h^3 sum'] -> (1/(2 pi^2)) h (-Z)
        assert C * 2.0 * math.pi ** 2 / h == pytest.approx(-zeta, rel=1e-4)


def test_bracket_falls_like_one_over_n():
    recip = synth.make_config("c2").recip()
    beta = 0.05
    c = {n: g.gamma_term(recip, (n, n, n), beta) for n in (2, 3, 4)}
    assert c[2] > c[3] > c[4] > 0.0
    assert 3 * c[3] == pytest.approx(2 * c[2], rel=2e-3)
    assert 4 * c[4] == pytest.approx(2 * c[2], rel=2e-3)


def test_apply_gamma_shifts_occupied_diagonal_only():
    rng = np.random.default_rng(3)
    V = rng.standard_normal((5, 5)) + 1j * rng.standard_normal((5, 5))
    W = g.apply_gamma(V, 2, 0.25)
    D = W - V
    assert np.array_equal(np.diag(D), np.array([-0.25, -0.25, 0, 0, 0]))
    D[np.diag_indices(5)] = 0
    assert not np.any(D)
