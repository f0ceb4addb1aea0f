"""Pins of the oracle's symmetrised Nyquist variant of the continuous Green
operator (eq. (15), operator "MSS"; reading: at a mode with some q_i = pi,
the mean of eq. (8) at q and at the grid partner of q) against what the
paper and the mathematics fix (no GPU).

* Where no component of q is pi, MSS is the continuous operator (eq. (8)).
* At the Nyquist modes it is real, has the minor and major symmetries of
  eq. (26), and takes equal values at a mode and its grid partner, so the
  Hermitian symmetry G(q)* = G(-q) that eq. (14) was introduced to restore
  holds on the grid and the inverse transform of G tau is real for a real
  tau (the paper's reason for eqs. (14)/(15)).
* On an x-laminate the field only has modes (m, 0, 0), where MSS is the
  exact one-dimensional projection even at the Nyquist mode (its own
  partner): the scheme reproduces the laminate's closed form for any layer
  thickness, while eq. (14)'s (C0)^-1 does so only for even thicknesses.
* The direct and accelerated schemes share the fixed point (§3) for the
  same reference medium, with eq. (43) summed off the Nyquist modes
  (reading R9: eq. (15) does not impose equilibrium there; over every mode
  eta stalls).  Unlike eq. (14), which imposes sigma(q) = 0 there, the mean
  of two C0-dependent operators makes the fixed point depend on C0.
"""
import itertools

import numpy as np
import pytest

import oracle as O
from microstructure import laminate, voronoi_cells

REF = O.Reference(0.7, 0.45)


def _partner(index, shape):
    return tuple((-i) % n for i, n in zip(index, shape))


def test_equals_the_continuous_operator_off_the_nyquist_modes():
    shape = (6, 8, 4)
    for index in [(1, 2, 3), (5, 7, 1), (2, 3, 0)]:
        a = O.green_tensor_at("MSS", REF, shape, index)
        b = O.green_tensor_at("MS", REF, shape, index)
        assert np.allclose(a, b, atol=1e-15)
        iz, iy, ix = index
        q = np.array([2 * np.pi * O.signed_modes(shape[2])[ix] / shape[2],
                      2 * np.pi * O.signed_modes(shape[1])[iy] / shape[1],
                      2 * np.pi * O.signed_modes(shape[0])[iz] / shape[0]])
        assert np.allclose(a, O.green_continuous_closed_form(REF, q), atol=1e-14)


def test_nyquist_modes_are_real_symmetric_and_equal_at_grid_partners():
    shape = (6, 8, 4)  # (nz, ny, nx): Nyquist indices 3, 4, 2
    nyq = []
    for index in itertools.product(range(6), range(8), range(4)):
        if index == (0, 0, 0):
            continue
        if index[0] == 3 or index[1] == 4 or index[2] == 2:
            nyq.append(index)
    assert len(nyq) > 20
    worst_change = 0.0
    for index in nyq:
        G = O.green_tensor_at("MSS", REF, shape, index)
        assert np.abs(G.imag).max() < 1e-15
        G = G.real
        assert np.allclose(G, G.transpose(1, 0, 2, 3), atol=1e-15)  # minor symmetries
        assert np.allclose(G, G.transpose(0, 1, 3, 2), atol=1e-15)
        assert np.allclose(G, G.transpose(2, 3, 0, 1), atol=1e-15)  # major symmetry, eq. (26)
        Gp = O.green_tensor_at("MSS", REF, shape, _partner(index, shape))
        assert np.allclose(Gp, np.conj(O.green_tensor_at("MSS", REF, shape, index)), atol=1e-15)
        # eq. (8) taken at q alone breaks this where the partner differs
        iz, iy, ix = index
        q = np.array([2 * np.pi * O.signed_modes(n)[i] / n for i, n in ((ix, 4), (iy, 8), (iz, 6))])
        worst_change = max(worst_change, np.abs(O.green_continuous_closed_form(REF, q) - G).max())
    assert worst_change > 1e-2  # the symmetrisation changes the operator there


def test_real_field_gives_a_real_strain(rng):
    shape = (6, 8, 4)
    t = rng.standard_normal((3, 3) + shape)
    t = 0.5 * (t + t.transpose(1, 0, 2, 3, 4))
    e = O.inverse_dft(O.green_apply("MSS", REF, O.forward_dft(t), shape))
    assert np.abs(e.imag).max() <= 1e-15 * np.abs(e.real).max()


@pytest.mark.parametrize("scheme", ["DS", "AS"])
def test_laminate_exact_for_odd_thickness(scheme):
    labels = np.array([1] * 3 + [0] * 5, dtype=np.uint8)  # odd layers on an even grid
    shape = (4, 6, 8)
    phase = laminate(shape, labels)
    E, nu = [1.0, 7.0], [0.3, 0.2]
    macro = [0.7, -0.3, 0.4, 0.2, -0.5, 0.6]
    exact = O.laminate_exact(labels, E, nu, macro)
    r = O.solve(phase, E, nu, macro, op="MSS", scheme=scheme, tol=1e-13, max_iter=3000)
    assert r.converged
    assert np.abs(r.eps - exact[:, :, None, None, :]).max() < 1e-11
    # eq. (14) on the same laminate: off by the Nyquist content of the layering
    r14 = O.solve(phase, E, nu, macro, op="MS", scheme=scheme, tol=1e-13, max_iter=3000)
    assert np.abs(r14.eps - exact[:, :, None, None, :]).max() > 1e-2


def test_direct_and_accelerated_schemes_share_the_fixed_point():
    phase, _, _ = voronoi_cells((6, 8, 10), 6, 3, 5)
    E, nu = [1.0, 5.0, 20.0], [0.2, 0.3, 0.35]
    macro = [0.3, -0.1, 0.2, 0.05, -0.2, 0.4]
    lam, mu = O.lame_from_young(E, nu)
    ref = O.reference_medium(lam, mu, "DS")
    a = O.solve(phase, E, nu, macro, op="MSS", scheme="AS", tol=1e-12, max_iter=3000, ref=ref)
    d = O.solve(phase, E, nu, macro, op="MSS", scheme="DS", tol=1e-12, max_iter=3000, ref=ref)
    assert a.converged and d.converged
    assert np.abs(a.eps - d.eps).max() < 1e-9
    # another reference medium, another fixed point (eq. (14): the same one)
    g = O.solve(phase, E, nu, macro, op="MSS", scheme="AS", tol=1e-12, max_iter=3000)
    assert np.abs(g.eps - a.eps).max() > 1e-3
    g14 = O.solve(phase, E, nu, macro, op="MS", scheme="AS", tol=1e-12, max_iter=3000)
    a14 = O.solve(phase, E, nu, macro, op="MS", scheme="AS", tol=1e-12, max_iter=3000, ref=ref)
    assert np.abs(g14.eps - a14.eps).max() < 1e-9
    # over every mode the residual of this fixed point stays large
    sig = O.homogenization.apply_phasewise([O.stiffness_tensor(l, m) for l, m in zip(lam, mu)], phase, a.eps)
    assert O.equilibrium_norm("MS", sig) > 1e-2
