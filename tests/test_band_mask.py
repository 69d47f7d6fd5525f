"""The Theta^MT band-pair criterion (Sec. III.D) on a constructed case.

Bands in irreducible representations A (3-fold), B (2-fold), A' (1) and C (2):
an operator with the full symmetry has matrix elements only within blocks of the
same representation (A with A', whose bands are not degenerate with A's), so
theta_mask must keep exactly those pairs. The example is built from the blocks,
then the bands are shuffled (the mask follows the bands, not their order).
"""
import numpy as np

from paper_1003_0524_amd import symmetry as sy


def test_theta_mask_recovers_representation_blocks():
    rng = np.random.default_rng(4)
    energies = np.array([-1.0, -1.0, -1.0, -0.5, -0.5, 0.2, 0.7, 0.7])
    rep = np.array(["A", "A", "A", "B", "B", "A", "C", "C"])
    nb = len(energies)
    theta = np.zeros((nb, nb), dtype=np.complex128)
    for i in range(nb):
        for j in range(nb):
            if rep[i] == rep[j]:
                theta[i, j] = rng.standard_normal() + 1j * rng.standard_normal()
    theta = (theta + theta.conj().T) / 2
    perm = rng.permutation(nb)
    mask = sy.theta_mask(theta[np.ix_(perm, perm)], energies[perm])
    expect = (rep[:, None] == rep[None, :])[np.ix_(perm, perm)]
    assert np.array_equal(mask, expect)
    # a tiny accidental element below the tolerance does not link representations
    theta2 = theta.copy()
    theta2[0, 3] = theta2[3, 0] = 1e-12
    assert np.array_equal(sy.theta_mask(theta2, energies), rep[:, None] == rep[None, :])
