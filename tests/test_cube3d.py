"""Cubic-inclusion cell of §5.2: the cell's construction, and the oracle
against the symmetry the paper states for each operator: sigma_12 of the
centred cube under the shear load is even under the three mirrors through
the cell centre for the continuous, centered and rotated operators (their
discrete problems keep the cell's mirror symmetry) and not for G^W, whose
one-sided differences break it."""
import numpy as np
import pytest

import oracle as O
from paper_1412_8398_amd import cube3d as Q


def test_cube_cell_and_section():
    for L in (8, 32, 256):
        ph = Q.cube_inclusion(L)
        assert ph.mean() == 0.125
        for a in range(3):
            assert np.array_equal(ph, np.flip(ph, axis=a))
    # the paper's plane x_3 = -0.2461 is the lower face of voxel plane 65 L / 256
    assert [Q.section_index(L) for L in (256, 512, 1024)] == [65, 130, 260]
    s = np.arange(16.0).reshape(4, 4)
    assert np.array_equal(Q.coarsen2(s), [[2.5, 4.5], [10.5, 12.5]])
    with pytest.raises(ValueError):
        Q.cube_inclusion(10)


@pytest.mark.parametrize("op,symmetric", [("MS", True), ("C", True), ("W", False), ("R", True)])
def test_oracle_mirror_symmetry_of_sigma12(op, symmetric):
    ph = Q.cube_inclusion(8)
    r = O.solve(ph, [Q.E1, Q.CHI * Q.E1], [Q.NU, Q.NU], list(Q.MACRO), op=op, scheme="AS", tol=1e-8,
                max_iter=5000)
    assert r.eta <= 1e-8
    s12 = O.tensor_to_voigt(r.sigma)[5]
    asym = max(np.abs(s12 - np.flip(s12, axis=a)).max() for a in range(3)) / np.abs(s12).max()
    if symmetric:
        assert asym < 1e-12
    else:
        assert asym > 0.1


def test_moduli_rate_helpers():
    """The §6.2 study's settling index and its rescaled Boolean medium (the
    same sphere centres at every resolution)."""
    from paper_1412_8398_amd import moduli_rate as M

    assert M.settle(np.array([2.0, 1.0, 1.02, 1.001, 1.0])) == 3
    assert M.settle(np.array([1.0, 1.0])) == 0
    _, a = M.medium(16)
    _, b = M.medium(32)
    assert a.n_spheres == b.n_spheres and np.allclose(b.centers, 2 * a.centers)
